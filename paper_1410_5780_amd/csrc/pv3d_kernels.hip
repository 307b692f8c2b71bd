// HIP kernels of libpv3d for gfx950 (MI355X): the per-sun shadow-map path of
// arXiv:1410.5780, Sec. 2 Steps 3-4.
//
// Per sun position:
//   setup       one workgroup per sun: image basis, window over the module
//               corners, depth range, per-module beam and depth bias, and the
//               mask of tiles that hold samples
//   tri_setup   one thread per triangle (and per module): FP64 light-space
//               transform, culling, guard-band clip, 1/256-texel snap,
//               fixed-point edge and depth planes; per-tile counts in LDS
//   bin_scan    exclusive scan of the tile counts (one workgroup)
//   bin_scatter triangle ids and modules into tile bins: per-workgroup LDS
//               ranks, one global atomic per (workgroup, tile)
//   tile        one workgroup per tile. Full route: 8x8-pixel stamps per
//               wave with whole-stamp reject / accept and ds_min_u32 into an
//               LDS depth tile, optional coalesced store. Sparse route: only
//               texels that hold a sample are evaluated. Either way the
//               samples whose texel lies in the tile are depth-checked there.
//   sample_test the same depth check from a materialised picture (one wave
//               per cell), kept as an independent second route
//   loss        one workgroup per sun: substring capacities, ideal bypass
//               string power, strings summed in order
//   energy      sum of power * dt in sun order
// (Triangle, tile) pairs are spread over the lanes of a wave, and tiles
// read triangle records in batches, so neither binning nor raster waits on
// one memory round trip per pair.
//
// Arithmetic: binary64 with contraction disabled (-ffp-contract=off), every
// dot product as (ax*bx + ay*by) + az*bz, so the FP64 steps give the same
// bits as any other IEEE implementation of the same formulas; everything
// after the snap is exact integer arithmetic.
#include "pv3d_device.h"

namespace pv3d {
namespace {

struct d3 {
    double x, y, z;
};

__device__ __forceinline__ d3 ld3(const double* p) { return d3{p[0], p[1], p[2]}; }
__device__ __forceinline__ double dot(d3 a, d3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
__device__ __forceinline__ d3 cross(d3 a, d3 b) {
    return d3{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ d3 add(d3 a, d3 b) { return d3{a.x + b.x, a.y + b.y, a.z + b.z}; }

__device__ __forceinline__ int64_t floor_shift(int64_t a, int s) { return a >> s; }  // arithmetic

// Load of a word that other workgroups of the same launch update with
// atomics: read at the device's coherence point, not from a cached copy.
template <typename T>
__device__ __forceinline__ T ld_dev(const T* p) {
    return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// ---------------------------------------------------------------------------
// generator preparation
// ---------------------------------------------------------------------------
__device__ __forceinline__ void module_corner(const Module& m, int q, d3& p) {
    d3 o = ld3(m.o), u = ld3(m.u), v = ld3(m.v);
    if (q == 0) p = o;
    else if (q == 1) p = add(o, u);
    else if (q == 2) p = add(add(o, u), v);
    else p = add(o, v);
}

// Axis-aligned box of the scene vertices and module corners: per-block partial
// min / max, then one block folds the partials into the bounding sphere.
__global__ __launch_bounds__(256) void k_bounds_partial(SceneDev sc, GenDev g, double* partial) {
    __shared__ double red[6][256];
    const int64_t n_pts = sc.n_vert + 4 * (int64_t)g.n_mod;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n_pts; i += (int64_t)gridDim.x * 256) {
        d3 p;
        if (i < sc.n_vert) p = ld3(sc.xyz + 3 * i);
        else module_corner(g.mods[(i - sc.n_vert) / 4], (int)((i - sc.n_vert) % 4), p);
        lo[0] = fmin(lo[0], p.x); lo[1] = fmin(lo[1], p.y); lo[2] = fmin(lo[2], p.z);
        hi[0] = fmax(hi[0], p.x); hi[1] = fmax(hi[1], p.y); hi[2] = fmax(hi[2], p.z);
    }
    for (int c = 0; c < 3; c++) {
        red[c][threadIdx.x] = lo[c];
        red[3 + c][threadIdx.x] = hi[c];
    }
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int c = 0; c < 3; c++) {
                red[c][threadIdx.x] = fmin(red[c][threadIdx.x], red[c][threadIdx.x + w]);
                red[3 + c][threadIdx.x] = fmax(red[3 + c][threadIdx.x], red[3 + c][threadIdx.x + w]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) partial[blockIdx.x * 6 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(64) void k_bounds_final(const double* partial, int32_t n_part, double* sphere) {
    if (threadIdx.x != 0) return;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int b = 0; b < n_part; b++)
        for (int c = 0; c < 3; c++) {
            lo[c] = fmin(lo[c], partial[b * 6 + c]);
            hi[c] = fmax(hi[c], partial[b * 6 + 3 + c]);
        }
    d3 ctr{(lo[0] + hi[0]) * 0.5, (lo[1] + hi[1]) * 0.5, (lo[2] + hi[2]) * 0.5};
    d3 dg{hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
    sphere[0] = ctr.x;
    sphere[1] = ctr.y;
    sphere[2] = ctr.z;
    sphere[3] = 0.5 * sqrt(dot(dg, dg));
}

// Fractional sample positions along a module edge: sample q (= k*cell + a) of
// k*n cells sits at (q + 1/2) / (k*n).
__global__ void k_sample_tables(double* fu, double* fv, int32_t k, int32_t n_cu, int32_t n_cv) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < k * n_cu) fu[i] = ((double)i + 0.5) / (double)(k * n_cu);
    if (i < k * n_cv) fv[i] = ((double)i + 0.5) / (double)(k * n_cv);
}

// ---------------------------------------------------------------------------
// per-sun view, module terms and the tiles that hold samples
// ---------------------------------------------------------------------------
__device__ __forceinline__ d3 to_light(const View& V, d3 p) {
    return d3{(dot(p, ld3(V.e1)) - V.ox) * V.itx, (dot(p, ld3(V.e2)) - V.oy) * V.ity,
              (dot(p, ld3(V.d)) - V.znear) * V.izd};
}

// A rectangle of tiles; empty when x0 > x1.
struct TileBox {
    int32_t x0, x1, y0, y1;
    __device__ int32_t count() const { return x0 > x1 ? 0 : (x1 - x0 + 1) * (y1 - y0 + 1); }
};

__device__ __forceinline__ TileBox rec_box(int32_t ilo, int32_t ihi, int32_t jlo, int32_t jhi, int32_t T) {
    return TileBox{ilo / T, ihi / T, jlo / T, jhi / T};
}

// Tile range of the texels a module's samples can fall in: the texel box of
// its corners widened by one texel, clamped to the map like the samples.
__device__ TileBox module_box(const View& V, const Module& M, int32_t n, int32_t T) {
    double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
    for (int q = 0; q < 4; q++) {
        d3 p;
        module_corner(M, q, p);
        d3 l = to_light(V, p);
        xmin = fmin(xmin, l.x); xmax = fmax(xmax, l.x);
        ymin = fmin(ymin, l.y); ymax = fmax(ymax, l.y);
    }
    const double hi = (double)(n - 1);
    int32_t i0 = (int32_t)fmin(fmax(floor(xmin) - 1.0, 0.0), hi), i1 = (int32_t)fmin(fmax(floor(xmax) + 1.0, 0.0), hi);
    int32_t j0 = (int32_t)fmin(fmax(floor(ymin) - 1.0, 0.0), hi), j1 = (int32_t)fmin(fmax(floor(ymax) + 1.0, 0.0), hi);
    return TileBox{i0 / T, i1 / T, j0 / T, j1 / T};
}

constexpr int kMaxMaskWords = 512;   // up to 16384 tiles per sun

struct SetupLds {
    double red[5][256];
    View sv;
    uint32_t mask[kMaxMaskWords];
    int any_front;
};

// One sun: sun3 is its unit vector, dn its DNI; view, beam_s, bias_s and
// tmask_s receive this sun's view, per-module beam and bias, and tile mask.
__device__ void setup_body(SetupLds& L, const double* sun3, double dn, const GenDev& g, const double* sphere,
                           int32_t n, View* view, double* beam_s, int32_t* bias_s, const TileGrid& tg,
                           uint32_t* tmask_s) {
    auto& red = L.red;
    auto& any_front = L.any_front;
    auto& sv = L.sv;
    auto& mask = L.mask;
    const int tid = threadIdx.x;
    const d3 sn = ld3(sun3);
    const bool up = sn.z > 0.0;
    if (tid == 0) any_front = 0;
    for (int q = tid; q < tg.words; q += 256) mask[q] = 0;
    __syncthreads();
    if (up)
        for (int m = tid; m < g.n_mod; m += 256)
            if (dot(ld3(g.mods[m].n), sn) > 0.0) any_front = 1;
    __syncthreads();
    const bool go = up && any_front;
    d3 d{-sn.x, -sn.y, -sn.z};
    d3 a = fabs(d.z) < 0.9 ? d3{0.0, 0.0, 1.0} : d3{1.0, 0.0, 0.0};
    d3 w = cross(a, d);
    double wl = sqrt(dot(w, w));
    d3 e1{w.x / wl, w.y / wl, w.z / wl};
    d3 e2 = cross(d, e1);
    double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY, zfar = -INFINITY;
    if (go)
        for (int m = tid; m < g.n_mod; m += 256)
            for (int q = 0; q < 4; q++) {
                d3 p;
                module_corner(g.mods[m], q, p);
                double u = dot(p, e1), v = dot(p, e2), z = dot(p, d);
                umin = fmin(umin, u); umax = fmax(umax, u);
                vmin = fmin(vmin, v); vmax = fmax(vmax, v);
                zfar = fmax(zfar, z);
            }
    red[0][tid] = umin; red[1][tid] = -umax; red[2][tid] = vmin; red[3][tid] = -vmax; red[4][tid] = -zfar;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (tid < k)
            for (int c = 0; c < 5; c++) red[c][tid] = fmin(red[c][tid], red[c][tid + k]);
        __syncthreads();
    }
    if (tid == 0) {
        View V;
        for (int c = 0; c < 3; c++) { V.e1[c] = 0; V.e2[c] = 0; V.d[c] = 0; }
        V.ox = V.oy = V.itx = V.ity = V.znear = V.izd = 0.0;
        V.valid = 0;
        V.pad = 0;
        if (go) {
            umin = red[0][0]; umax = -red[1][0]; vmin = red[2][0]; vmax = -red[3][0]; zfar = -red[4][0];
            double su = umax - umin, svv = vmax - vmin;
            if (su > 0.0 && svv > 0.0) {
                V.e1[0] = e1.x; V.e1[1] = e1.y; V.e1[2] = e1.z;
                V.e2[0] = e2.x; V.e2[1] = e2.y; V.e2[2] = e2.z;
                V.d[0] = d.x; V.d[1] = d.y; V.d[2] = d.z;
                V.itx = (double)(n - 2) / su;
                V.ity = (double)(n - 2) / svv;
                V.ox = umin - su / (double)(n - 2);
                V.oy = vmin - svv / (double)(n - 2);
                d3 c = ld3(sphere);
                V.znear = dot(c, d) - sphere[3];
                V.izd = (double)kDepthMax / (zfar - V.znear);
                V.valid = 1;
            }
        }
        sv = V;
        *view = V;
    }
    __syncthreads();
    for (int m = tid; m < g.n_mod; m += 256) {
        d3 nh = ld3(g.mods[m].n);
        double cm = dot(nh, sn);
        double bm = 0.0;
        int32_t bi = -1;
        if (up) {
            bm = cm > 0.0 ? dn * cm : 0.0;
            if (cm > 0.0 && sv.valid) {
                double nx = dot(nh, ld3(sv.e1)), ny = dot(nh, ld3(sv.e2)), nz = dot(nh, ld3(sv.d));
                double gxs = (fabs(nx / nz) * sv.izd) / sv.itx;
                double gys = (fabs(ny / nz) * sv.izd) / sv.ity;
                double b = ceil((0.5 + 1.0 / 512.0) * (gxs + gys)) + 2.0;
                if (!(b <= (double)kDepthMax)) b = (double)kDepthMax;
                bi = (int32_t)b;
            }
        }
        beam_s[m] = bm;
        bias_s[m] = bi;
        if (tmask_s && bi >= 0) {
            const TileBox b = module_box(sv, g.mods[m], n, tg.tile);
            for (int32_t ty = b.y0; ty <= b.y1; ty++)
                for (int32_t tx = b.x0; tx <= b.x1; tx++) {
                    const int32_t q = ty * tg.ntx + tx;
                    atomicOr(&mask[q >> 5], 1u << (q & 31));
                }
        }
    }
    if (tmask_s) {
        __syncthreads();
        for (int q = tid; q < tg.words; q += 256) tmask_s[q] = mask[q];
    }
}

__global__ __launch_bounds__(256) void k_setup(const double* sun, const double* dni, GenDev g,
                                               const double* sphere, int32_t n, View* views,
                                               double* beam, int32_t* bias, TileGrid tg, uint32_t* tmask) {
    __shared__ SetupLds L;
    const int64_t s = blockIdx.x;
    GenDev gs = g;                                    // trackers: this sun's posed modules
    if (g.mods_sun) gs.mods = g.mods_sun + s * g.n_mod;
    setup_body(L, sun + 3 * s, dni[s], gs, sphere, n, views + s, beam + s * g.n_mod, bias + s * g.n_mod, tg,
               tmask ? tmask + s * tg.words : nullptr);
}

// Trackers (Sec. 3.4; the reading taken is ideal tracking, no angle limits,
// no backtracking): every module of a tracker keeps its coordinates in the
// tracker's frame, which turns with the sun. Rest frame u0 = a x z, v0 = a,
// n0 = z (a: horizontal unit axis); for sun s
//   kind 1: v' = a, n' = unit(s - (s.a) a), u' = v' x n'
//   kind 2: n' = s, u' = unit(z x s) (u0 at the zenith), v' = n' x u'.
// One thread per (sun, module); suns below the horizon and modules of no
// tracker keep the rest pose. The front normal is recomputed from the posed
// edges with the operations the generator definition uses.
__device__ __forceinline__ d3 unit3(d3 v) {
    const double l = sqrt(dot(v, v));
    return d3{v.x / l, v.y / l, v.z / l};
}

__device__ __forceinline__ d3 in_frame(double c0, double c1, double c2, d3 u, d3 v, d3 n) {
    return d3{(c0 * u.x + c1 * v.x) + c2 * n.x, (c0 * u.y + c1 * v.y) + c2 * n.y, (c0 * u.z + c1 * v.z) + c2 * n.z};
}

__global__ __launch_bounds__(256) void k_pose(const double* sun, int64_t n_sun, const Module* rest, int32_t n_mod,
                                              const TrackerDev* trk, const int32_t* mod_trk, Module* posed) {
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n_sun * n_mod) return;
    const int64_t s = i / n_mod;
    const int32_t m = (int32_t)(i % n_mod);
    Module M = rest[m];
    const int32_t t = mod_trk[m];
    const d3 sv = ld3(sun + 3 * s);
    if (t >= 0 && sv.z > 0.0) {
        const TrackerDev& T = trk[t];
        const d3 z{0.0, 0.0, 1.0}, a = ld3(T.a), P = ld3(T.p);
        d3 u, v, n;
        if (T.kind == 1) {
            const double sa = dot(sv, a);
            const d3 q{sv.x - sa * a.x, sv.y - sa * a.y, sv.z - sa * a.z};
            v = a;
            n = dot(q, q) > 1e-30 ? unit3(q) : z;
            u = cross(v, n);
        } else {
            const d3 h = cross(z, sv);
            n = sv;
            u = dot(h, h) > 1e-30 ? unit3(h) : cross(a, z);
            v = cross(n, u);
        }
        const d3 u0 = cross(a, z), v0 = a, n0 = z;
        const d3 r{M.o[0] - P.x, M.o[1] - P.y, M.o[2] - P.z};
        const d3 o = add(P, in_frame(dot(r, u0), dot(r, v0), dot(r, n0), u, v, n));
        const d3 U0 = ld3(M.u), W0 = ld3(M.v);
        const d3 U = in_frame(dot(U0, u0), dot(U0, v0), dot(U0, n0), u, v, n);
        const d3 W = in_frame(dot(W0, u0), dot(W0, v0), dot(W0, n0), u, v, n);
        const double cx = U.y * W.z - U.z * W.y, cy = U.z * W.x - U.x * W.z, cz = U.x * W.y - U.y * W.x;
        const double l = sqrt((cx * cx + cy * cy) + cz * cz);
        M.o[0] = o.x; M.o[1] = o.y; M.o[2] = o.z;
        M.u[0] = U.x; M.u[1] = U.y; M.u[2] = U.z;
        M.v[0] = W.x; M.v[1] = W.y; M.v[2] = W.z;
        M.n[0] = cx / l; M.n[1] = cy / l; M.n[2] = cz / l;
    }
    posed[i] = M;
}

// Bounding sphere from a box given by value (centre, half diagonal), in
// stream order with the kernels that read it.
__global__ void k_box_sphere(double lx, double ly, double lz, double hx, double hy, double hz, double* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double dx = hx - lx, dy = hy - ly, dz = hz - lz;
    out[0] = (lx + hx) * 0.5;
    out[1] = (ly + hy) * 0.5;
    out[2] = (lz + hz) * 0.5;
    out[3] = 0.5 * sqrt((dx * dx + dy * dy) + dz * dz);
}

// ---------------------------------------------------------------------------
// triangle set-up and binning
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool mask_has(const uint32_t* m, int32_t q) {
    return m == nullptr || ((m[q >> 5] >> (q & 31)) & 1u);
}

// Edges of a set-up triangle as the binning test needs them.
struct Edges {
    int64_t e0[3];
    int32_t a[3], b[3];
    int32_t ilo, ihi, jlo, jhi;
};

// False when one edge excludes every pixel centre of the triangle's box
// clipped to tile (tx, ty): that tile cannot hold a covered pixel.
__device__ __forceinline__ bool tile_overlap(const Edges& E, int32_t tx, int32_t ty, int32_t T) {
    const int32_t i0 = max(E.ilo, tx * T), i1 = min(E.ihi, tx * T + T - 1);
    const int32_t j0 = max(E.jlo, ty * T), j1 = min(E.jhi, ty * T + T - 1);
    for (int e = 0; e < 3; e++) {
        const int64_t A = (int64_t)E.a[e] * 256, B = (int64_t)E.b[e] * 256;
        if (E.e0[e] + A * (A > 0 ? i1 : i0) + B * (B > 0 ? j1 : j0) < 0) return false;
    }
    return true;
}

__device__ __forceinline__ void edges_of(const TriRec& r, Edges& E) {
    for (int e = 0; e < 3; e++) { E.e0[e] = r.e0[e]; E.a[e] = r.a[e]; E.b[e] = r.b[e]; }
    E.ilo = r.ilo; E.ihi = r.ihi; E.jlo = r.jlo; E.jhi = r.jhi;
}

// Every (lane, tile) pair of a wave, 64 at a time: lane L owns the tiles of
// box[L] (kind 0: none, 1: a triangle whose tiles pass the overlap test,
// 2: a module, every tile of its box). f(q, payload of the owner) runs for
// each kept tile q on the lane that takes the pair. All lanes of the wave
// must call this (the shuffles need every lane active).
template <typename F>
__device__ __forceinline__ void wave_pairs(const TileBox& box, int32_t kind, const Edges& E, int32_t payload, int lane,
                                           int32_t T, int32_t ntx, const uint32_t* mask, F&& f) {
    const int32_t cnt = kind ? box.count() : 0;
    int32_t incl = cnt;
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t v = __shfl_up(incl, off, 64);
        if (lane >= off) incl += v;
    }
    const int32_t total = __shfl(incl, 63, 64);
    const int32_t excl = incl - cnt;
    for (int32_t base = 0; base < total; base += 64) {
        const bool live = base + lane < total;
        const int32_t p = min(base + lane, total - 1);
        int32_t lo = 0, hi = 63;                       // owner: last lane whose first pair is <= p
        for (int it = 0; it < 6; it++) {
            const int32_t mid = (lo + hi + 1) >> 1;
            const bool le = __shfl(excl, mid, 64) <= p;
            lo = le ? mid : lo;
            hi = le ? hi : mid - 1;
        }
        const int32_t o = lo;
        const int32_t okind = __shfl(kind, o, 64);
        const int32_t ox0 = __shfl(box.x0, o, 64), ox1 = __shfl(box.x1, o, 64), oy0 = __shfl(box.y0, o, 64);
        const int32_t q = p - __shfl(excl, o, 64);
        const int32_t bw = ox1 - ox0 + 1;
        const int32_t ty = oy0 + q / bw, tx = ox0 + q % bw;
        Edges oe;
        for (int e = 0; e < 3; e++) {
            oe.e0[e] = __shfl(E.e0[e], o, 64);
            oe.a[e] = __shfl(E.a[e], o, 64);
            oe.b[e] = __shfl(E.b[e], o, 64);
        }
        oe.ilo = __shfl(E.ilo, o, 64); oe.ihi = __shfl(E.ihi, o, 64);
        oe.jlo = __shfl(E.jlo, o, 64); oe.jhi = __shfl(E.jhi, o, 64);
        const int32_t opay = __shfl(payload, o, 64);
        const int32_t tq = ty * ntx + tx;
        bool keep = live && mask_has(mask, tq);
        if (keep && okind == 1) keep = tile_overlap(oe, tx, ty, T);
        if (keep) f(tq, opay);
    }
}

// Exclusive prefix sum of v over the 256 threads of a workgroup; total gets
// the sum. Every thread calls it (it holds two barriers).
__device__ __forceinline__ int32_t block_scan_excl(int32_t v, int32_t* wsum, int32_t& total, int lane, int wv) {
    int32_t x = v;
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    int32_t base = 0;
    total = 0;
    for (int w = 0; w < 4; w++) {
        const int32_t t = wsum[w];
        base += w < wv ? t : 0;
        total += t;
    }
    __syncthreads();
    return base + x - v;
}

// The XCD the wave runs on.
__device__ __forceinline__ int32_t xcc_id() { return (int32_t)__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20); }

// Lanes of the wave below this one whose bit is set.
__device__ __forceinline__ int32_t lanes_below(unsigned long long bal) {
    return (int32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
}

// floor(q / k) for 0 <= q < 2^32 / k: the high word of q m with m = ceil(2^32 / k).
// With m = (2^32 + e) / k, 0 <= e < k, the product carries an excess of q e / 2^32 < 1
// over q / k, too little to reach the next integer (k = 1: m = 0 marks the identity).
struct DivK {
    uint32_t m;
};
__device__ __forceinline__ DivK div_by(int32_t k) {
    return DivK{k > 1 ? (uint32_t)((0x100000000ull + (unsigned long long)(k - 1)) / (unsigned long long)k) : 0u};
}
__device__ __forceinline__ int32_t div_k(DivK d, int32_t q) {
    return d.m ? (int32_t)__umulhi((uint32_t)q, d.m) : q;
}

// Relaxed device-scope atomics on device memory (the count and flag arrays),
// issued as global rather than flat instructions: a flat access may address
// LDS, so it also holds the LDS counter, and the next wait for an LDS result
// (a shuffle, a staged triangle) would wait for the atomic's round trip.
typedef __attribute__((address_space(1))) uint32_t global_u32;
__device__ __forceinline__ void dev_add(uint32_t* p, uint32_t v) {
    __hip_atomic_fetch_add((global_u32*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void dev_or(uint32_t* p, uint32_t v) {
    __hip_atomic_fetch_or((global_u32*)p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Last index i in [0, n) with key(a[i]) <= x, for keys that do not decrease
// and key(a[0]) <= x.
template <int SHIFT>
__device__ __forceinline__ int32_t last_at_most(const uint32_t* a, int32_t n, uint32_t x) {
    int32_t lo = 0, hi = n - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if ((a[mid] >> SHIFT) <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Snap, orient and set up one light-space triangle and append its record;
// returns the record id, or -1 when it covers no pixel centre.
__device__ int32_t emit_triangle(const d3 t[3], int32_t n, const BinBuffers& bb, SunCounters* ctr, Edges& E,
                                 bool& large) {
    int64_t X[3], Y[3];
    double Z[3];
    const double tv[3][3] = {{t[0].x, t[0].y, t[0].z}, {t[1].x, t[1].y, t[1].z}, {t[2].x, t[2].y, t[2].z}};
    for (int q = 0; q < 3; q++) {
        X[q] = (int64_t)floor(tv[q][0] * 256.0 + 0.5);
        Y[q] = (int64_t)floor(tv[q][1] * 256.0 + 0.5);
        Z[q] = tv[q][2];
    }
    int64_t A = (X[1] - X[0]) * (Y[2] - Y[0]) - (X[2] - X[0]) * (Y[1] - Y[0]);
    if (A == 0) return -1;
    if (A < 0) {
        int64_t tx = X[1]; X[1] = X[2]; X[2] = tx;
        int64_t ty = Y[1]; Y[1] = Y[2]; Y[2] = ty;
        double tz = Z[1]; Z[1] = Z[2]; Z[2] = tz;
        A = -A;
    }
    int64_t xmin = min(X[0], min(X[1], X[2])), xmax = max(X[0], max(X[1], X[2]));
    int64_t ymin = min(Y[0], min(Y[1], Y[2])), ymax = max(Y[0], max(Y[1], Y[2]));
    // pixel centres (256 i + 128) inside the snapped box, clipped to the map
    int64_t ilo = -floor_shift(-(xmin - 128), kSubBits), ihi = floor_shift(xmax - 128, kSubBits);
    int64_t jlo = -floor_shift(-(ymin - 128), kSubBits), jhi = floor_shift(ymax - 128, kSubBits);
    ilo = max(ilo, (int64_t)0); jlo = max(jlo, (int64_t)0);
    ihi = min(ihi, (int64_t)n - 1); jhi = min(jhi, (int64_t)n - 1);
    if (ilo > ihi || jlo > jhi) return -1;

    TriRec r;
    const int ea[3] = {1, 2, 0}, eb[3] = {2, 0, 1};
    for (int e = 0; e < 3; e++) {
        int64_t xa = X[ea[e]], ya = Y[ea[e]];
        int64_t dx = X[eb[e]] - xa, dy = Y[eb[e]] - ya;
        bool tl = (dy < 0) || (dy == 0 && dx < 0);
        // E(P) = dx (Py - ya) - dy (Px - xa) at P = (128, 128), pixel (0, 0)
        int64_t e00 = dx * (128 - ya) - dy * (128 - xa);
        r.e0[e] = e00 - (tl ? 0 : 1);
        r.a[e] = (int32_t)(-dy);
        r.b[e] = (int32_t)dx;
    }
    double Ad = (double)A / 65536.0;
    double dx1 = (double)(X[1] - X[0]) / 256.0, dy1 = (double)(Y[1] - Y[0]) / 256.0;
    double dx2 = (double)(X[2] - X[0]) / 256.0, dy2 = (double)(Y[2] - Y[0]) / 256.0;
    double dz1 = Z[1] - Z[0], dz2 = Z[2] - Z[0];
    double gx = (dz1 * dy2 - dz2 * dy1) / Ad;
    double gy = (dx1 * dz2 - dx2 * dz1) / Ad;
    const double GLIM = 1073741824.0;
    gx = fmin(fmax(gx, -GLIM), GLIM);
    gy = fmin(fmax(gy, -GLIM), GLIM);
    int64_t i0 = floor_shift(xmin, kSubBits), j0 = floor_shift(ymin, kSubBits);
    i0 = min(max(i0, (int64_t)0), (int64_t)n - 1);
    j0 = min(max(j0, (int64_t)0), (int64_t)n - 1);
    double za = (Z[0] + gx * (((double)i0 + 0.5) - (double)X[0] / 256.0))
                + gy * (((double)j0 + 0.5) - (double)Y[0] / 256.0);
    const double ZLIM = 1099511627776.0;
    za = fmin(fmax(za, -ZLIM), ZLIM);
    int64_t gxf = (int64_t)floor(gx * 65536.0 + 0.5);
    int64_t gyf = (int64_t)floor(gy * 65536.0 + 0.5);
    int64_t zaf = (int64_t)floor(za * 65536.0 + 0.5);
    r.z0 = zaf - i0 * gxf - j0 * gyf;
    r.gx = gxf;
    r.gy = gyf;
    r.ilo = (int16_t)ilo; r.ihi = (int16_t)ihi; r.jlo = (int16_t)jlo; r.jhi = (int16_t)jhi;

    int32_t idx = atomicAdd(&ctr->n_rec, 1);
    if (idx >= bb.rec_cap) {
        atomicOr(&ctr->overflow, 1);
        return -1;
    }
    bb.rec[idx] = r;
    edges_of(r, E);
    large = rec_box((int32_t)ilo, (int32_t)ihi, (int32_t)jlo, (int32_t)jhi, bb.tile).count() > bb.large_tiles;
    if (large) {
        int32_t li = atomicAdd(&ctr->n_large, 1);
        bb.large[li] = idx;
    }
    return idx;
}

// Sutherland-Hodgman against one side of the guard square.
__device__ int clip_side(const d3* in, int nin, d3* out, int axis, double c, bool keep_ge) {
    int m = 0;
    for (int q = 0; q < nin; q++) {
        d3 p = in[q], r = in[(q + 1) % nin];
        double pa = axis == 0 ? p.x : p.y, ra = axis == 0 ? r.x : r.y;
        bool pin = keep_ge ? (pa >= c) : (pa <= c);
        bool rin = keep_ge ? (ra >= c) : (ra <= c);
        if (pin) out[m++] = p;
        if (pin != rin) {
            double t = (c - pa) / (ra - pa);
            d3 o{p.x + (r.x - p.x) * t, p.y + (r.y - p.y) * t, p.z + (r.z - p.z) * t};
            if (axis == 0) o.x = c;
            else o.y = c;
            out[m++] = o;
        }
    }
    return m;
}

// A triangle reaching beyond the guard square: clip, fan, set up each piece
// and count it (one lane; such triangles are rare).
// Pair mode: write item k (first pair s, c pairs) and mark the chunks whose
// first pair it holds.
__device__ __forceinline__ void put_pair_item(const BinBuffers& bb, SunCounters* ctr, unsigned long long at,
                                              int32_t c, int32_t id, const TileBox& box) {
    const int64_t k = (int64_t)(at >> 32), s = (int64_t)(at & 0xFFFFFFFFull);
    // the capacities bound every sun (an item per record and module, at most
    // as many pairs as bin entries); were one exceeded, every item below
    // item_cap is still written and the pair passes read no pair past bin_cap
    if (k >= bb.item_cap || s + c > bb.bin_cap) atomicOr(&ctr->overflow, 1);
    if (k >= bb.item_cap) return;
    bb.pitems[k] = PairItem{id, (int32_t)min(s, (int64_t)bb.bin_cap), (uint32_t)box.x0 | ((uint32_t)box.x1 << 16),
                            (uint32_t)box.y0 | ((uint32_t)box.y1 << 16)};
    const int64_t e = min(s + c, (int64_t)bb.bin_cap);
    for (int64_t q = (s + kPairChunk - 1) / kPairChunk; q * kPairChunk < e; q++) bb.pchunk[q] = (int32_t)k;
}

// Pair mode, every thread of the workgroup: the threads with c > 0 pairs
// take consecutive items and pair ranges, with one 64-bit atomic (items in
// the high word, pairs in the low) per workgroup, so that item starts grow
// with the item index. lds holds 5 words.
__device__ void reserve_pair_items(unsigned long long* lds, const BinBuffers& bb, SunCounters* ctr, int32_t c,
                                   int32_t id, const TileBox& box, int lane, int wv) {
    const unsigned long long v = c > 0 ? ((1ull << 32) | (unsigned long long)c) : 0ull;
    unsigned long long x = v;
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) lds[wv] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long tot = lds[0] + lds[1] + lds[2] + lds[3];
        lds[4] = tot ? atomicAdd(bb.pctr, tot) : 0ull;
    }
    __syncthreads();
    unsigned long long at = lds[4] + x - v;
    for (int w = 0; w < wv; w++) at += lds[w];
    __syncthreads();
    if (c > 0) put_pair_item(bb, ctr, at, c, id, box);
}

__device__ __noinline__ void clip_and_emit(d3 t0, d3 t1, d3 t2, int32_t n, const BinBuffers& bb, SunCounters* ctr,
                                           uint32_t* cnt, const uint32_t* mask) {
    d3 a[8], b[8];
    a[0] = t0; a[1] = t1; a[2] = t2;
    int m = clip_side(a, 3, b, 0, -kGuard, true);
    if (m < 3) return;
    m = clip_side(b, m, a, 0, kGuard, false);
    if (m < 3) return;
    m = clip_side(a, m, b, 1, -kGuard, true);
    if (m < 3) return;
    m = clip_side(b, m, a, 1, kGuard, false);
    if (m < 3) return;
    for (int q = 1; q + 1 < m; q++) {
        d3 f[3] = {a[0], a[q], a[q + 1]};
        Edges E;
        bool large = false;
        const int32_t rid = emit_triangle(f, n, bb, ctr, E, large);
        if (rid < 0 || large) continue;
        const TileBox box = rec_box(E.ilo, E.ihi, E.jlo, E.jhi, bb.tile);
        if (bb.pitems) {                                   // pair mode: an item of its own
            const int32_t c = box.count();
            if (c > 0) put_pair_item(bb, ctr, atomicAdd(bb.pctr, (1ull << 32) | (unsigned long long)c), c, rid, box);
            continue;
        }
        for (int32_t ty = box.y0; ty <= box.y1; ty++)
            for (int32_t tx = box.x0; tx <= box.x1; tx++) {
                const int32_t tq = ty * bb.ntx + tx;
                if (mask_has(mask, tq) && tile_overlap(E, tx, ty, bb.tile)) atomicAdd(&cnt[tq], 1u);
            }
    }
}

// True when every triangle of scene block blk would be culled for this view:
// the block's vertex box, mapped to light space corner by corner, lies beyond
// the far depth or wholly outside the window by more than a texel. The
// per-triangle test sees each vertex's own mapping, which differs from the
// corners' convex combination by rounding many orders of magnitude below the
// margin, so the skip never drops a triangle the test would keep.
__device__ __forceinline__ bool block_culled(const View& V, const double* cbox, int64_t blk, int32_t n) {
    const double* b = cbox + 6 * blk;
    double x0 = INFINITY, x1 = -INFINITY, y0 = INFINITY, y1 = -INFINITY, z0 = INFINITY;
    for (int q = 0; q < 8; q++) {
        const d3 l = to_light(V, d3{b[(q & 1) ? 3 : 0], b[(q & 2) ? 4 : 1], b[(q & 4) ? 5 : 2]});
        x0 = fmin(x0, l.x); x1 = fmax(x1, l.x);
        y0 = fmin(y0, l.y); y1 = fmax(y1, l.y);
        z0 = fmin(z0, l.z);
    }
    auto mg = [](double v) { return 1.0 + 1e-9 * fabs(v); };
    return z0 > (double)kDepthMax + mg(z0) || x1 < -mg(x1) || x0 >= (double)n + mg(x0) || y1 < -mg(y1) ||
           y0 >= (double)n + mg(y0);
}

// Triangles [t0, t1) of the set-up index space (scene triangles, module
// triangles, modules); t0 is a multiple of kTriBlock. In pair mode
// (bb.pitems set) the binned records and module boxes only take their items
// in pair space, and cnt holds the 5 words of the reservation. Otherwise,
// 256 at a time, the per-tile counts of the pairs are accumulated in LDS
// (cnt, n_tiles words) and added to the global counts once; with cnt ==
// nullptr every pair goes straight to the global counts.
__device__ void tri_setup_body(uint32_t* cnt, int64_t t0, int64_t t1, const View& V, const SceneDev& sc,
                               const GenDev& g, const int32_t* bias_s, int32_t n, const BinBuffers& bb,
                               SunCounters* ctr_s, const uint32_t* tmask_s) {
    const int64_t n_tri_all = sc.n_tri + (g.occluders ? 2 * (int64_t)g.n_mod : 0);
    const int lane = threadIdx.x & 63;
    if (!V.valid) {                                   // nothing is drawn or tested for this sun
        for (int64_t t = t0 + threadIdx.x; t < t1; t += 256)
            if (t >= n_tri_all && t < n_tri_all + g.n_mod) bb.modbox[t - n_tri_all] = make_int4(1, 0, 1, 0);
        return;
    }
    if (sc.cbox && t1 <= sc.n_tri) {                   // scene triangles only: leave if every block is culled
        bool all = true;
        for (int64_t tb = t0; tb < t1 && all; tb += kTriBlock) all = block_culled(V, sc.cbox, tb / kTriBlock, n);
        if (all) return;
    }
    const bool pairs = bb.pitems != nullptr;
    uint32_t* gcnt = reinterpret_cast<uint32_t*>(bb.tile_count);
    if (cnt && !pairs) {
        for (int32_t q = threadIdx.x; q < bb.n_tiles; q += 256) cnt[q] = 0;
        __syncthreads();
    }
    uint32_t* sink = cnt ? cnt : gcnt;
    static_assert(kTriBlock == 256, "one thread per triangle of a block");
    for (int64_t tb = t0; tb < t1; tb += 256) {
        const int64_t t = tb + threadIdx.x;
        const bool skip = sc.cbox && tb < sc.n_tri && block_culled(V, sc.cbox, tb / kTriBlock, n);
        TileBox box{1, 0, 1, 0};
        int32_t kind = 0, pid = 0;
        Edges E;
        for (int e = 0; e < 3; e++) { E.e0[e] = 0; E.a[e] = 0; E.b[e] = 0; }
        E.ilo = E.ihi = E.jlo = E.jhi = 0;
        if (t < t1 && t < n_tri_all) {
            if (!(skip && t < sc.n_tri)) {
                d3 c[3];
                if (t < sc.n_tri) {
                    for (int q = 0; q < 3; q++) c[q] = ld3(sc.xyz + 3 * (int64_t)sc.tri[3 * t + q]);
                } else {
                    int64_t mt = t - sc.n_tri;
                    const Module& M = g.mods[mt / 2];
                    module_corner(M, 0, c[0]);
                    if ((mt & 1) == 0) { module_corner(M, 1, c[1]); module_corner(M, 2, c[2]); }
                    else { module_corner(M, 2, c[1]); module_corner(M, 3, c[2]); }
                }
                d3 l[3];
                for (int q = 0; q < 3; q++) l[q] = to_light(V, c[q]);
                double zmin = fmin(l[0].z, fmin(l[1].z, l[2].z));
                double xmin = fmin(l[0].x, fmin(l[1].x, l[2].x)), xmax = fmax(l[0].x, fmax(l[1].x, l[2].x));
                double ymin = fmin(l[0].y, fmin(l[1].y, l[2].y)), ymax = fmax(l[0].y, fmax(l[1].y, l[2].y));
                bool keep = !(zmin > (double)kDepthMax) && !(xmax < 0.0 || xmin >= (double)n || ymax < 0.0 || ymin >= (double)n);
                if (keep) {
                    bool big = false;
                    for (int q = 0; q < 3; q++)
                        if (fabs(l[q].x) >= kGuard || fabs(l[q].y) >= kGuard) big = true;
                    if (big) {
                        clip_and_emit(l[0], l[1], l[2], n, bb, ctr_s, sink, tmask_s);
                    } else {
                        bool large = false;
                        const int32_t rid = emit_triangle(l, n, bb, ctr_s, E, large);
                        if (rid >= 0 && !large) {
                            box = rec_box(E.ilo, E.ihi, E.jlo, E.jhi, bb.tile);
                            kind = 1;
                            pid = rid;
                        }
                    }
                }
            }
        } else if (t < t1 && t < n_tri_all + g.n_mod) {
            const int32_t m = (int32_t)(t - n_tri_all);
            TileBox b{1, 0, 1, 0};
            if (bias_s[m] >= 0) b = module_box(V, g.mods[m], n, bb.tile);
            bb.modbox[m] = make_int4(b.x0, b.x1, b.y0, b.y1);
            if (b.count() > 0) { box = b; kind = 2; pid = -(m + 1); }
        }
        if (pairs)
            reserve_pair_items(reinterpret_cast<unsigned long long*>(cnt), bb, ctr_s, kind ? box.count() : 0, pid, box,
                               lane, threadIdx.x >> 6);
        else
            wave_pairs(box, kind, E, 0, lane, bb.tile, bb.ntx, tmask_s,
                       [&](int32_t tq, int32_t) { atomicAdd(&sink[tq], 1u); });
    }
    if (cnt && !pairs) {
        __syncthreads();
        for (int32_t q = threadIdx.x; q < bb.n_tiles; q += 256)
            if (cnt[q]) atomicAdd(&gcnt[q], cnt[q]);
    }
}

// Group form: blockIdx.y picks the sun of the group.
__global__ __launch_bounds__(256) void k_tri_setup_g(const SunGroup* __restrict__ grp, const View* views, SceneDev sc,
                                                     const int32_t* bias, int32_t n, SunCounters* ctr) {
    extern __shared__ uint32_t cnt[];
    const GroupSun& S = grp->sun[blockIdx.y];
    const int64_t total = sc.n_tri + (S.g.occluders ? 2 * (int64_t)S.g.n_mod : 0) + S.g.n_mod;
    const int64_t t0 = blockIdx.x * 256ll;
    tri_setup_body(cnt, t0, min(t0 + 256, total), views[S.s], sc, S.g, bias + S.s * S.g.n_mod, n, S.bb, ctr + S.s,
                   S.tmask);
}

// Exclusive prefix sum over the NT threads of a workgroup (wave shuffles,
// then the wave totals); total gets the sum. Every thread calls it; wsum
// holds NT / 64 words.
template <int NT>
__device__ __forceinline__ unsigned long long scan_excl64(unsigned long long v, unsigned long long* wsum,
                                                          unsigned long long& total) {
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    unsigned long long x = v;
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned long long y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    unsigned long long base = 0;
    total = 0;
    for (int w = 0; w < NT / 64; w++) {
        const unsigned long long t = wsum[w];
        base += w < wv ? t : 0ull;
        total += t;
    }
    __syncthreads();
    return base + x - v;
}

// Exclusive scan of the tile counts by NT threads; every count is left at
// zero for the next sun. With list != nullptr the tiles holding at least one
// entry are also listed as work items and their number returned (every
// thread): in tile order when split_at < 0, otherwise the most entries first
// (entries bucketed by eight), a tile with more than split_at > 0 entries as
// its four quadrants. part holds 2 NT + 2 kScanBuckets ints; the count total
// is left in part[0].
constexpr int kScanBuckets = 256;
// Tiles with fewer than 8 kLightBuckets bin entries (the last kLightBuckets
// buckets of the heaviest-first order, so the tail of the work list) are
// light: the group tile kernel takes them one wave each.
constexpr int kLightBuckets = 6;

// A thread with at most kScanKeep tiles keeps their counts in registers for
// the later passes instead of reading the starts back from memory (C2 year
// 335 -> 328 ms). kept_at(kept, j) is kept[j], read without a variable index
// so that the array stays in registers.
constexpr int kScanKeep = 8;

// slot[key] += w for every lane with ok, the lanes of a wave that share a key
// with one atomic between them; each such lane gets the slot's value before
// its own share (lanes of one key in lane order). key < 2^BITS, w is 1 or 4.
// The lanes that share a key are found one key bit at a time (a ballot per
// bit), so the cost does not grow with the number of distinct keys in the
// wave; the first lane of every key then adds for its group, all groups in
// one atomic instruction on distinct slots. Every lane of the wave calls it.
template <int BITS>
__device__ __forceinline__ int32_t wave_add(int32_t* slot, bool ok, int32_t key, int32_t w) {
    unsigned long long peers = __ballot(ok);
#pragma unroll
    for (int b = 0; b < BITS; b++) {
        const unsigned long long set = __ballot((key >> b) & 1);
        peers &= ((key >> b) & 1) ? set : ~set;
    }
    const unsigned long long four = peers & __ballot(w != 1);
    const unsigned long long one = peers & ~four;
    const int32_t before = lanes_below(one) + 4 * lanes_below(four);
    const int32_t total = __popcll(one) + 4 * __popcll(four);
    const int leader = peers ? __ffsll((long long)peers) - 1 : 0;
    const int lane = threadIdx.x & 63;
    int32_t base = 0;
    if (ok && lane == leader) base = atomicAdd(&slot[key], total);
    base = __shfl(base, leader, 64);
    return ok ? base + before : 0;
}

template <int KEEP>
__device__ __forceinline__ int32_t kept_at(const int32_t (&kept)[KEEP], int32_t j) {
    int32_t c = 0;
#pragma unroll
    for (int32_t q = 0; q < KEEP; q++) c = q == j ? kept[q] : c;
    return c;
}

template <int NT, bool COHERENT, int KEEP = kScanKeep>
__device__ int32_t scan_body(int32_t* part, int32_t n_tiles, const BinBuffers& bb, int32_t* list, int32_t split_at) {
    static_assert(NT >= kScanBuckets && NT % 64 == 0, "a thread per bucket");
    static_assert(kScanBuckets == 256, "bucket keys take eight bits");
    const int tid = threadIdx.x;
    unsigned long long* wsum = reinterpret_cast<unsigned long long*>(part + 2);
    const int32_t per = (n_tiles + NT - 1) / NT;
    const int32_t b0 = min(tid * per, n_tiles), b1 = min(b0 + per, n_tiles);
    const bool keep = per <= KEEP;
    int32_t kept[KEEP];
    int32_t sum = 0, nz = 0;
    if (keep) {
#pragma unroll
        for (int32_t j = 0; j < KEEP; j++) {
            const int32_t i = b0 + j;
            kept[j] = i < b1 ? (COHERENT ? ld_dev(bb.tile_count + i) : bb.tile_count[i]) : 0;
            sum += kept[j];
            nz += kept[j] > 0 ? 1 : 0;
        }
    } else {
        for (int32_t i = b0; i < b1; i++) {
            const int32_t c = COHERENT ? ld_dev(bb.tile_count + i) : bb.tile_count[i];
            sum += c;
            nz += c > 0 ? 1 : 0;
        }
    }
    // entries and non-empty tiles, scanned together
    unsigned long long tot;
    const unsigned long long ex =
        scan_excl64<NT>(((unsigned long long)nz << 32) | (unsigned long long)(uint32_t)sum, wsum, tot);
    const bool in_order = list && split_at < 0;
    int32_t run = (int32_t)(uint32_t)ex, lpos = (int32_t)(ex >> 32);
    for (int32_t i = b0; i < b1; i++) {
        const int32_t c = keep ? kept_at<KEEP>(kept, i - b0) : (COHERENT ? ld_dev(bb.tile_count + i) : bb.tile_count[i]);
        bb.tile_start[i] = run;
        if (COHERENT) {       // words other units update with atomics are written with atomics only
            __hip_atomic_store(bb.tile_cursor + i, run, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(bb.tile_count + i, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            bb.tile_cursor[i] = run;
            bb.tile_count[i] = 0;
        }
        if (in_order && c > 0) list[lpos++] = (i << 3) | kWholeTile;
        run += c;
    }
    const int32_t n_entries = (int32_t)(uint32_t)tot, n_nonempty = (int32_t)(tot >> 32);
    if (tid == NT - 1) bb.tile_start[n_tiles] = n_entries;
    if (tid == 0) part[0] = n_entries;
    __syncthreads();
    if (!list || in_order) return n_nonempty;
    // heaviest first: counting sort of the non-empty tiles by entry bucket. The tiles of
    // one picture often share a few buckets, so the lanes of a wave with the same bucket
    // take one atomic together (one per lane serialised about 120 us per sun of 16,384 tiles)
    int32_t* hist = part + 2 * NT;
    int32_t* cur = hist + kScanBuckets;
    for (int q = tid; q < kScanBuckets; q += NT) hist[q] = 0;
    __syncthreads();
    for (int32_t j = 0; j < per; j++) {               // the same trip count on every lane
        const int32_t i = b0 + j;
        const int32_t c = i < b1 ? (keep ? kept_at<KEEP>(kept, j) : bb.tile_start[i + 1] - bb.tile_start[i]) : 0;
        const int32_t bk = kScanBuckets - 1 - min(c >> 3, kScanBuckets - 1);
        (void)wave_add<8>(hist, c > 0, bk, (split_at > 0 && c > split_at) ? 4 : 1);
    }
    __syncthreads();
    const unsigned long long own = tid < kScanBuckets ? (unsigned long long)hist[tid] : 0ull;
    unsigned long long n_items64;
    const unsigned long long first = scan_excl64<NT>(own, wsum, n_items64);
    if (tid < kScanBuckets) cur[tid] = (int32_t)first;
    if (tid == kScanBuckets - kLightBuckets) part[1] = (int32_t)first;   // light tiles are the list's tail
    const int32_t n_items = (int32_t)n_items64;
    __syncthreads();
    for (int32_t j = 0; j < per; j++) {
        const int32_t i = b0 + j;
        const int32_t c = i < b1 ? (keep ? kept_at<KEEP>(kept, j) : bb.tile_start[i + 1] - bb.tile_start[i]) : 0;
        const int32_t bk = kScanBuckets - 1 - min(c >> 3, kScanBuckets - 1);
        const bool split = split_at > 0 && c > split_at;
        const int32_t pos = wave_add<8>(cur, c > 0, bk, split ? 4 : 1);
        if (c > 0) {
            if (split)
                for (int32_t q = 0; q < 4; q++) list[pos + q] = (i << 3) | q;
            else
                list[pos] = (i << 3) | kWholeTile;
        }
    }
    __syncthreads();
    return n_items;
}

// One workgroup per sun of a group. NT x KEEP tiles stay in registers: 512 x 8 up to
// 4,096 tiles (64-texel tiles of a 4096 picture; 512 threads find room on a CU beside
// the other lane's tile pass sooner than 1024), 1024 x 16 up to 16,384 (of an 8192
// picture, where re-reading the starts from memory made the scan take 83 us).
template <int NT, int KEEP>
__global__ __launch_bounds__(NT) void k_bin_scan_g(const SunGroup* __restrict__ grp, int32_t n_tiles) {
    __shared__ __attribute__((aligned(16))) int32_t part[2 * NT + 2 * kScanBuckets];
    const BinBuffers& bb = grp->sun[blockIdx.x].bb;
    const int32_t n_items = scan_body<NT, false, KEEP>(part, n_tiles, bb, bb.tile_list, bb.split_at);
    if (bb.tile_list && threadIdx.x == 0) {
        bb.list_ctr[0] = n_items;
        bb.list_ctr[1] = 0;
        bb.list_ctr[2] = bb.split_at >= 0 ? part[1] : n_items;   // first light item
        for (int j = 0; j < kXcds; j++) bb.list_ctr[kXcdStride * (j + 1)] = 0;
    }
}

// Item of the scatter: a binned triangle record (kind 1) or a module (kind 2).
__device__ __forceinline__ void scatter_item(int32_t item, int32_t n_rec, int32_t n_items, const BinBuffers& bb,
                                             TileBox& box, int32_t& kind, Edges& E, int32_t& id) {
    box = TileBox{1, 0, 1, 0};
    kind = 0;
    id = 0;
    for (int e = 0; e < 3; e++) { E.e0[e] = 0; E.a[e] = 0; E.b[e] = 0; }
    E.ilo = E.ihi = E.jlo = E.jhi = 0;
    if (item >= n_items) return;
    if (item < n_rec) {
        const TriRec& r = bb.rec[item];
        edges_of(r, E);
        const TileBox b = rec_box(r.ilo, r.ihi, r.jlo, r.jhi, bb.tile);
        id = item;
        if (b.count() <= bb.large_tiles) { box = b; kind = 1; }
        return;
    }
    const int32_t m = item - n_rec;
    const int4 v = bb.modbox[m];
    id = -(m + 1);
    box = TileBox{v.x, v.y, v.z, v.w};
    if (box.count() > 0) kind = 2;
}

// A contiguous range of items per unit (unit u of n_units): count per tile
// in LDS, take one block of bin slots per (unit, tile) with a single global
// atomic, then place every (item, tile) pair at its LDS-assigned rank inside
// that block. The pair filter is the one the triangle set-up counted with.
// With lds == nullptr every pair takes its slot with its own global atomic.
__device__ void scatter_body(uint32_t* lds, int32_t unit, int32_t n_units, const BinBuffers& bb, int32_t n_mod,
                             int32_t n_rec_all, SunCounters* ctr_s, const uint32_t* tmask_s) {
    const int lane = threadIdx.x & 63;
    const int32_t n_rec = min(n_rec_all, bb.rec_cap);
    const int32_t total = n_rec + n_mod;
    const int32_t per = (total + n_units - 1) / n_units;
    const int32_t i0 = unit * per, i1 = min(i0 + per, total);
    if (i0 >= i1) return;
    if (!lds) {
        for (int32_t it0 = i0; it0 < i1; it0 += 256) {
            TileBox box;
            int32_t kind, id;
            Edges E;
            scatter_item(it0 + (int32_t)threadIdx.x, n_rec, i1, bb, box, kind, E, id);
            wave_pairs(box, kind, E, id, lane, bb.tile, bb.ntx, tmask_s, [&](int32_t tq, int32_t oid) {
                const uint32_t pos = (uint32_t)atomicAdd(&bb.tile_cursor[tq], 1);
                if (pos < (uint32_t)bb.bin_cap) bb.bins[pos] = oid;
                else atomicOr(&ctr_s->overflow, 1);
            });
        }
        return;
    }
    uint32_t* cnt = lds;                 // per-tile count, then running rank
    uint32_t* base = lds + bb.n_tiles;   // per-tile first bin slot of this unit
    for (int32_t q = threadIdx.x; q < bb.n_tiles; q += 256) cnt[q] = 0;
    __syncthreads();
    for (int32_t it0 = i0; it0 < i1; it0 += 256) {
        TileBox box;
        int32_t kind, id;
        Edges E;
        scatter_item(it0 + (int32_t)threadIdx.x, n_rec, i1, bb, box, kind, E, id);
        wave_pairs(box, kind, E, id, lane, bb.tile, bb.ntx, tmask_s, [&](int32_t tq, int32_t) { atomicAdd(&cnt[tq], 1u); });
    }
    __syncthreads();
    for (int32_t q = threadIdx.x; q < bb.n_tiles; q += 256) {
        const uint32_t c = cnt[q];
        if (c) base[q] = (uint32_t)atomicAdd(&bb.tile_cursor[q], (int32_t)c);
        cnt[q] = 0;
    }
    __syncthreads();
    for (int32_t it0 = i0; it0 < i1; it0 += 256) {
        TileBox box;
        int32_t kind, id;
        Edges E;
        scatter_item(it0 + (int32_t)threadIdx.x, n_rec, i1, bb, box, kind, E, id);
        wave_pairs(box, kind, E, id, lane, bb.tile, bb.ntx, tmask_s, [&](int32_t tq, int32_t oid) {
            const uint32_t pos = base[tq] + atomicAdd(&cnt[tq], 1u);
            if (pos < (uint32_t)bb.bin_cap) bb.bins[pos] = oid;
            else atomicOr(&ctr_s->overflow, 1);
        });
    }
}

// Pair mode: every pair of the sun's pair space, in chunks of kPairChunk over
// the grid. A thread finds its item among the (at most kPairChunk) items the
// chunk touches by binary search over their starts in LDS, then its tile;
// f(tile, id) runs for the pairs the binning keeps: tiles with samples, and
// for a record only the tiles its edges reach (the filter of wave_pairs).
template <typename F>
__device__ void pair_chunk(const BinBuffers& bb, const uint32_t* tmask, uint32_t* st, int64_t q, int64_t n_items,
                           int64_t n_pairs, F&& f) {
    const int32_t nty = bb.n_tiles / bb.ntx;
    static_assert(kPairChunk == 256, "one thread per pair of a chunk");
    const int32_t k0 = bb.pchunk[q];
    const bool k0_ok = k0 >= 0 && k0 < n_items;
    const int64_t k = k0 + (int64_t)threadIdx.x;
    st[threadIdx.x] = (k0_ok && k < n_items) ? (uint32_t)bb.pitems[k].start : 0xFFFFFFFFu;
    __syncthreads();
    const int64_t p = q * kPairChunk + threadIdx.x;
    if (k0_ok && p < n_pairs && st[0] <= (uint32_t)p) {
        const PairItem it = bb.pitems[k0 + last_at_most<0>(st, kPairChunk, (uint32_t)p)];
        const int32_t x0 = (int32_t)(it.xr & 0xFFFFu), x1 = (int32_t)(it.xr >> 16);
        const int32_t y0 = (int32_t)(it.yr & 0xFFFFu);
        const int32_t r = (int32_t)(p - it.start), bw = x1 - x0 + 1;
        const int32_t tx = x0 + (bw > 0 ? r % bw : 0), ty = y0 + (bw > 0 ? r / bw : 0);
        const int32_t tq = ty * bb.ntx + tx;
        bool keep = bw > 0 && tx < bb.ntx && ty < nty && it.id < bb.rec_cap;
        keep = keep && mask_has(tmask, tq);
        if (keep && it.id >= 0) {
            Edges E;
            edges_of(bb.rec[it.id], E);
            keep = tile_overlap(E, tx, ty, bb.tile);
        }
        if (keep) f(tq, it.id);
    }
    __syncthreads();
}

// A sun's item and pair counts, bounded by its buffers: a sun whose items
// overflowed them is reported by the host and evaluated no further; its
// reads stay inside the buffers all the same.
__device__ __forceinline__ void pair_space(const BinBuffers& bb, int64_t& n_items, int64_t& n_pairs) {
    const unsigned long long pc = *bb.pctr;
    n_items = min((int64_t)(pc >> 32), (int64_t)bb.item_cap);
    n_pairs = min((int64_t)(pc & 0xFFFFFFFFull), (int64_t)bb.bin_cap);
}

// Every chunk of every sun of a group, one sequence over the grid: chunk Q
// of the concatenated pair spaces belongs to the sun whose range holds it.
template <typename F>
__device__ void group_pair_chunks(const SunGroup* grp, uint32_t* st, long long* first, F&& f) {
    const int32_t ng = grp->n;
    if (threadIdx.x == 0) {
        long long acc = 0;
        for (int32_t q = 0; q < ng; q++) {
            int64_t ni, np;
            pair_space(grp->sun[q].bb, ni, np);
            first[q] = acc;
            acc += (np + kPairChunk - 1) / kPairChunk;
        }
        first[ng] = acc;
    }
    __syncthreads();
    const long long total = first[ng];
    for (long long Q = blockIdx.x; Q < total; Q += gridDim.x) {
        int32_t q = 0;
        while (q + 1 < ng && first[q + 1] <= Q) q++;
        q = __builtin_amdgcn_readfirstlane(q);
        const GroupSun& S = grp->sun[q];
        int64_t ni, np;
        pair_space(S.bb, ni, np);
        pair_chunk(S.bb, S.tmask, st, Q - first[q], ni, np, [&](int32_t tq, int32_t id) { f(S.bb, tq, id); });
    }
}

__global__ __launch_bounds__(256) void k_pair_count_g(const SunGroup* __restrict__ grp) {
    __shared__ uint32_t st[kPairChunk];
    __shared__ long long first[kMaxGroup + 1];
    group_pair_chunks(grp, st, first, [&](const BinBuffers& bb, int32_t tq, int32_t) { atomicAdd(&bb.tile_count[tq], 1); });
}

__global__ __launch_bounds__(256) void k_pair_scatter_g(const SunGroup* __restrict__ grp) {
    __shared__ uint32_t st[kPairChunk];
    __shared__ long long first[kMaxGroup + 1];
    group_pair_chunks(grp, st, first, [&](const BinBuffers& bb, int32_t tq, int32_t id) {
        const int32_t at = atomicAdd(&bb.tile_cursor[tq], 1);
        if (at < bb.bin_cap) bb.bins[at] = id;
    });
}

// ---------------------------------------------------------------------------
// tile kernel. Every tile gathers the modules whose samples may fall in it.
// Full route: raster every triangle into an LDS depth tile (the nearest depth
// wins, Fig. 3), optionally store the tile, then depth-check the samples
// whose texel lies in the tile (Fig. 4). Sparse route: the depth picture only
// matters at texels that hold a sample, so the tile lists those samples
// (sorted by texel row) and every triangle is tested at their texel centres
// only; a sample's shaded flag is the same as with the full picture.
// ---------------------------------------------------------------------------
constexpr int kMaxTileMods = 256;       // module entries kept in LDS per tile
constexpr int kMaxCellCounters = 256;   // per-wave cell counters of the full route
constexpr int kMaxTileCells = 1024;     // (module slot, cell) counters of the sparse route

struct TileCtx {
    int32_t x0, y0, n, bs, be, n_large;
    const TriRec* lrec;     // the first n_lrec records of the large list, kept in LDS
    int32_t n_lrec;
    const double* ftab;     // sample fractions, k n_cu along edge_u then k n_cv along edge_v, in LDS (when lds)
    const double* fu_g;     // the same fractions in device memory
    const double* fv_g;
    int32_t knu;
    bool lds;
};

// A sample's fractions along edge_u and edge_v. The two sources are read on
// separate branches, so that each load keeps its own address space.
__device__ __forceinline__ double frac_u(const TileCtx& c, int32_t qa) { return c.lds ? c.ftab[qa] : c.fu_g[qa]; }
__device__ __forceinline__ double frac_v(const TileCtx& c, int32_t qb) {
    return c.lds ? c.ftab[c.knu + qb] : c.fv_g[qb];
}

// Sample fractions (k n_cu along edge_u, then k n_cv along edge_v) a workgroup
// of the group tile kernel keeps in LDS when they fit.
constexpr int kFracCache = 256;

// Records of a sun's large list (triangles every tile checks) that a
// workgroup of the group tile kernel keeps in LDS while it takes that sun's
// tiles: the list is the same for every tile, and reading its records from
// memory for each tile was a large part of the tile pass on the rooftop
// workload (about 21 large triangles per tile).
constexpr int kLargeCache = 32;
// Light tiles a wave claims at a time. A sun's light tiles form kXcds strided
// sub-lists with a counter each (128 bytes apart): the waves of an XCD claim
// from their own sub-list, then help with the others. With one counter for every
// wave of the launch its device-scope atomics, not the tiles' work, set the
// pace when waves claimed tile by tile; each claim's round trip also stalls its
// wave, and large claims leave waves idle at the end of a short list. A claim
// takes one tile per kLightPerClaim tiles of the sub-list (rounded up), at least
// kLightClaimMin and at most kLightClaimMax: 5 on the rooftop (about 1,100
// light tiles per sub-list and sun), 2 on the row plant (about 180).
constexpr int32_t kLightPerClaim = 256;
constexpr int32_t kLightClaimMin = 2;
constexpr int32_t kLightClaimMax = 16;

// Triangle slots a wave of a light tile stages: kLargeCache + 8 kLightBuckets - 1
// candidates at most.
constexpr int kWaveSlots = 80;

// Waves take triangles in chunks; the lanes of the wave load the chunk's
// records at once, then the wave walks them one by one from registers.
constexpr int kChunk = 16;

struct RecLane {
    uint32_t w[20];
};

__device__ __forceinline__ int32_t next_chunk(int32_t* next, int lane) {
    int32_t got = 0;
    if (lane == 0) got = atomicAdd(next, kChunk);
    return __builtin_amdgcn_readfirstlane(got);
}

__device__ __forceinline__ int32_t load_chunk(const BinBuffers& bb, int32_t base, int32_t cnt, int32_t n_large,
                                              int32_t bs, int lane, RecLane& L) {
    for (int q = 0; q < 20; q++) L.w[q] = 0;
    int32_t rid = -1;
    if (lane < cnt) {
        const int32_t item = base + lane;
        rid = item < n_large ? bb.large[item] : bb.bins[bs + item - n_large];
        if (rid >= 0) {
            const uint4* p = reinterpret_cast<const uint4*>(bb.rec + rid);
            for (int q = 0; q < 5; q++) {
                const uint4 v = p[q];
                L.w[4 * q] = v.x; L.w[4 * q + 1] = v.y; L.w[4 * q + 2] = v.z; L.w[4 * q + 3] = v.w;
            }
        }
    }
    return rid;
}

__device__ __forceinline__ TriRec rec_of_lane(const RecLane& L, int i) {
    uint32_t w[20];
    for (int q = 0; q < 20; q++) w[q] = __builtin_amdgcn_readlane(L.w[q], i);
    TriRec r;
    __builtin_memcpy(&r, w, sizeof(TriRec));
    return r;
}

// A square of texels [x, x + size) x [y, y + size) inside a tile.
struct Rect {
    int32_t x, y, size;
};

// Per-module light-space affine map of the samples.
struct ModMap {
    d3 p0, du, dv;
};

__device__ __forceinline__ void module_map(const View& V, const Module& M, ModMap& mm) {
    const d3 e1 = ld3(V.e1), e2 = ld3(V.e2), dd = ld3(V.d);
    mm.p0 = to_light(V, ld3(M.o));
    const d3 U = ld3(M.u), W = ld3(M.v);
    mm.du = d3{dot(U, e1) * V.itx, dot(U, e2) * V.ity, dot(U, dd) * V.izd};
    mm.dv = d3{dot(W, e1) * V.itx, dot(W, e2) * V.ity, dot(W, dd) * V.izd};
}


// Light-space extent of a rect for sample selection: texels clamp to the map,
// so at a map border the rect reaches to infinity.
__device__ __forceinline__ void rect_bounds(const Rect& r, int32_t n, double& xl, double& xh, double& yl, double& yh) {
    xl = r.x == 0 ? -INFINITY : (double)r.x;
    xh = r.x + r.size >= n ? INFINITY : (double)(r.x + r.size);
    yl = r.y == 0 ? -INFINITY : (double)r.y;
    yh = r.y + r.size >= n ? INFINITY : (double)(r.y + r.size);
}

// Conservative range of sample rows qb whose texels can fall in the rect:
// the rect's corners mapped back to module coordinates (all rows when the
// map is nearly singular or the rect is open-ended).
__device__ __forceinline__ void row_range(const ModMap& mm, int32_t knv, double xl, double xh, double yl, double yh,
                                          int32_t& qb0, int32_t& qb1) {
    qb0 = 0;
    qb1 = knv - 1;
    const d3 du = mm.du, dv = mm.dv;
    const double det = du.x * dv.y - du.y * dv.x;
    if (!(fabs(det) > 1e-9 * (fabs(du.x * dv.y) + fabs(du.y * dv.x)) && det != 0.0)) return;
    if (!(isfinite(xl) && isfinite(xh) && isfinite(yl) && isfinite(yh))) return;
    double vmin = INFINITY, vmax = -INFINITY;
    const double cx[2] = {xl, xh}, cy[2] = {yl, yh};
    for (int qx = 0; qx < 2; qx++)
        for (int qy = 0; qy < 2; qy++) {
            const double fv = (du.x * (cy[qy] - mm.p0.y) - du.y * (cx[qx] - mm.p0.x)) / det;
            vmin = fmin(vmin, fv);
            vmax = fmax(vmax, fv);
        }
    const double b0 = floor(vmin * knv - 0.5) - 1.0, b1 = ceil(vmax * knv - 0.5) + 1.0;
    qb0 = (int32_t)fmax(b0, 0.0);
    qb1 = (int32_t)fmin(b1, (double)(knv - 1));
}

// Conservative column range [qa0, qa1] of one sample row whose texels can
// fall in the rect: the row is a line in light space; intersect it with the
// rect's slab in x and in y (widened by one sample for rounding).
__device__ __forceinline__ void col_range(const ModMap& mm, double fv, int32_t knu, double xl, double xh, double yl,
                                          double yh, int32_t& qa0, int32_t& qa1) {
    double lo = 0.0, hi = 1.0;
    const double bx = mm.p0.x + fv * mm.dv.x, by = mm.p0.y + fv * mm.dv.y;
    const double cs[2] = {mm.du.x, mm.du.y}, bs[2] = {bx, by}, ls[2] = {xl, yl}, hs[2] = {xh, yh};
    for (int q = 0; q < 2; q++) {
        const double c = cs[q], b = bs[q];
        if (fabs(c) > 1e-300) {
            double f0 = (ls[q] - 1.0 - b) / c, f1 = (hs[q] + 1.0 - b) / c;   // one texel of margin
            if (f0 > f1) { const double t = f0; f0 = f1; f1 = t; }
            lo = fmax(lo, f0);
            hi = fmin(hi, f1);
        } else if (!(b >= ls[q] - 1.0 && b <= hs[q] + 1.0)) {
            lo = 1.0; hi = 0.0;
        }
    }
    if (!(lo <= hi)) { qa0 = 1; qa1 = 0; return; }
    const double a0 = floor(lo * knu - 0.5) - 1.0, a1 = ceil(hi * knu - 0.5) + 1.0;
    qa0 = (int32_t)fmax(a0, 0.0);
    qa1 = (int32_t)fmin(a1, (double)(knu - 1));
}

// Texel and depth of sample (qa, qb), exactly as the definition computes
// them; false when its texel is not in the rect. zs is the sample depth
// clamped to int32 (the shaded test compares it with values below 2^25).
__device__ __forceinline__ bool sample_in_rect(const ModMap& mm, double fu, double fv, const Rect& r, int32_t n,
                                               int32_t* li, int32_t* lj, int32_t* zs) {
    const double x = (mm.p0.x + fu * mm.du.x) + fv * mm.dv.x;
    const double y = (mm.p0.y + fu * mm.du.y) + fv * mm.dv.y;
    const double z = (mm.p0.z + fu * mm.du.z) + fv * mm.dv.z;
    const double hi = (double)(n - 1);
    const int32_t i = (int32_t)fmin(fmax(floor(x), 0.0), hi);
    const int32_t j = (int32_t)fmin(fmax(floor(y), 0.0), hi);
    if (i < r.x || i >= r.x + r.size || j < r.y || j >= r.y + r.size) return false;
    *li = i - r.x;
    *lj = j - r.y;
    *zs = (int32_t)fmin(fmax(floor(z), -2147483648.0), 2147483647.0);
    return true;
}

// Record of a triangle touching the tile, with its box clipped to the tile;
// false when the box or an edge excludes the whole clipped box.
struct TriClip {
    int32_t ilo, ihi, jlo, jhi;
    int64_t EA[3], EB[3];
};

__device__ __forceinline__ bool clip_to_tile(const TriRec& R, int32_t x0, int32_t y0, int32_t TS, TriClip& t) {
    t.ilo = max((int32_t)R.ilo, x0); t.ihi = min((int32_t)R.ihi, x0 + TS - 1);
    t.jlo = max((int32_t)R.jlo, y0); t.jhi = min((int32_t)R.jhi, y0 + TS - 1);
    if (t.ilo > t.ihi || t.jlo > t.jhi) return false;
    bool outside = false;
    for (int e = 0; e < 3; e++) {
        t.EA[e] = (int64_t)R.a[e] * 256;
        t.EB[e] = (int64_t)R.b[e] * 256;
        const int64_t bmax = R.e0[e] + t.EA[e] * (t.EA[e] > 0 ? t.ihi : t.ilo) + t.EB[e] * (t.EB[e] > 0 ? t.jhi : t.jlo);
        outside |= bmax < 0;
    }
    return !outside;
}

// e0 + a x + b y for x = 256 i, y = 256 j (i, j texel offsets, so x and y fit
// 32 bits): each product is one 32 x 32 -> 64-bit multiply-add, and the sum
// is the exact value the 64-bit per-texel steps a 256, b 256 give.
__device__ __forceinline__ int64_t edge_at(int64_t e0, int32_t a, int32_t b, int32_t x, int32_t y) {
    return e0 + (int64_t)a * x + (int64_t)b * y;
}

// The record's box clipped to the rect; false when the box or an edge
// excludes the whole clipped box (the edge steps of t are not filled).
__device__ __forceinline__ bool clip_to_rect(const TriRec& R, const Rect& r, TriClip& t) {
    t.ilo = max((int32_t)R.ilo, r.x); t.ihi = min((int32_t)R.ihi, r.x + r.size - 1);
    t.jlo = max((int32_t)R.jlo, r.y); t.jhi = min((int32_t)R.jhi, r.y + r.size - 1);
    if (t.ilo > t.ihi || t.jlo > t.jhi) return false;
    bool outside = false;
    for (int e = 0; e < 3; e++) {
        const int64_t bmax = edge_at(R.e0[e], R.a[e], R.b[e], 256 * (R.a[e] > 0 ? t.ihi : t.ilo),
                                     256 * (R.b[e] > 0 ? t.jhi : t.jlo));
        outside |= bmax < 0;
    }
    return !outside;
}

__device__ __forceinline__ uint32_t depth_q(int64_t z) {
    const int64_t zq = z >> 16;
    return zq < 0 ? 0u : (zq > (int64_t)kDepthMax ? kDepthMax : (uint32_t)zq);
}

// Full raster of the tile's triangles into zt (all waves; `next` starts at 0).
template <int TS>
__device__ void raster_full(uint32_t* zt, int32_t* next, const BinBuffers& bb, const TileCtx& c, int lane) {
    constexpr int PITCH = TS + 8;
    const int32_t total = c.n_large + (c.be - c.bs);
    const int lx = lane & 7, ly = lane >> 3;
    for (;;) {
        const int32_t base = next_chunk(next, lane);
        if (base >= total) break;
        const int32_t cnt = min(kChunk, total - base);
        RecLane L;
        const int32_t rid = load_chunk(bb, base, cnt, c.n_large, c.bs, lane, L);
        for (int ci = 0; ci < cnt; ci++) {
        if (__builtin_amdgcn_readlane(rid, ci) < 0) continue;   // a module entry
        const TriRec R = rec_of_lane(L, ci);
        TriClip t;
        if (!clip_to_tile(R, c.x0, c.y0, TS, t)) continue;
        int64_t er[3], emaxo[3], emino[3], el[3];
        for (int e = 0; e < 3; e++) {
            emaxo[e] = (t.EA[e] > 0 ? 7 * t.EA[e] : 0) + (t.EB[e] > 0 ? 7 * t.EB[e] : 0);
            emino[e] = (t.EA[e] < 0 ? 7 * t.EA[e] : 0) + (t.EB[e] < 0 ? 7 * t.EB[e] : 0);
        }
        const int32_t sx0 = c.x0 + ((t.ilo - c.x0) & ~7), sy0 = c.y0 + ((t.jlo - c.y0) & ~7);
        for (int e = 0; e < 3; e++) {
            el[e] = t.EA[e] * lx + t.EB[e] * ly;
            er[e] = R.e0[e] + t.EA[e] * sx0 + t.EB[e] * sy0;
        }
        const int64_t gx = R.gx, gy = R.gy;
        const int64_t zl = gx * lx + gy * ly;
        int64_t zr = R.z0 + gx * sx0 + gy * sy0;
        for (int32_t sy = sy0; sy <= t.jhi; sy += 8) {
            int64_t es0 = er[0], es1 = er[1], es2 = er[2], zs = zr;
            const int32_t row = (sy - c.y0 + ly) * PITCH + lx;
            for (int32_t sx = sx0; sx <= t.ihi; sx += 8) {
                const bool skip = (es0 + emaxo[0] < 0) | (es1 + emaxo[1] < 0) | (es2 + emaxo[2] < 0);
                if (!skip) {
                    const bool full = (es0 + emino[0] >= 0) & (es1 + emino[1] >= 0) & (es2 + emino[2] >= 0);
                    const uint32_t D = depth_q(zs + zl);
                    bool cov = full;
                    if (!full) cov = ((es0 + el[0]) | (es1 + el[1]) | (es2 + el[2])) >= 0;
                    if (cov) atomicMin(&zt[row + (sx - c.x0)], D);
                }
                es0 += 8 * t.EA[0]; es1 += 8 * t.EA[1]; es2 += 8 * t.EA[2];
                zs += 8 * gx;
            }
            er[0] += 8 * t.EB[0]; er[1] += 8 * t.EB[1]; er[2] += 8 * t.EB[2];
            zr += 8 * gy;
        }
        }
    }
}

template <int TS>
__device__ void store_tile(const uint32_t* zt, uint32_t* map, const TileCtx& c, int tid) {
    constexpr int PITCH = TS + 8;
    const int32_t n = c.n;
    if ((n & 3) == 0) {
        for (int q = tid; q < TS * TS / 4; q += 256) {
            const int r = q / (TS / 4), cc = (q % (TS / 4)) * 4;
            const int32_t py = c.y0 + r, px = c.x0 + cc;
            if (py < n && px < n) {
                uint4 v;
                v.x = zt[r * PITCH + cc]; v.y = zt[r * PITCH + cc + 1];
                v.z = zt[r * PITCH + cc + 2]; v.w = zt[r * PITCH + cc + 3];
                *reinterpret_cast<uint4*>(map + (int64_t)py * n + px) = v;
            }
        }
    } else {
        for (int q = tid; q < TS * TS; q += 256) {
            const int r = q / TS, cc = q % TS;
            const int32_t py = c.y0 + r, px = c.x0 + cc;
            if (py < n && px < n) map[(int64_t)py * n + px] = zt[r * PITCH + cc];
        }
    }
}

// Depth check of the samples whose texel lies in rect r against the full LDS
// tile (waves over modules; each sample row gets its exact column range).
template <int TS>
__device__ void samples_full(const uint32_t* zt, const int32_t* mods, int32_t nm, bool mods_in_lds, uint32_t* cc,
                             const View& V, const BinBuffers& bb, const GenDev& g, const int32_t* bias,
                             const double* fu_tab, const double* fv_tab, int32_t k, const TileOut& out,
                             const TileCtx& c, const Rect& r, int lane, int wv) {
    constexpr int PITCH = TS + 8;
    const int32_t cpm = g.n_cu * g.n_cv;
    const int32_t knu = k * g.n_cu, knv = k * g.n_cv;
    const int32_t kk = k * k, words = (kk + 31) / 32;
    const bool lds_cells = cpm <= kMaxCellCounters;
    double xl, xh, yl, yh;
    rect_bounds(r, c.n, xl, xh, yl, yh);
    for (int32_t mi = wv; mi < nm; mi += 4) {
        int32_t m;
        if (!mods_in_lds) {
            const int32_t id = bb.bins[c.bs + mi];
            if (id >= 0) continue;
            m = -id - 1;
        } else {
            m = mods[mi];
        }
        const int32_t bm = bias[m];
        if (bm < 0) continue;
        ModMap mm;
        module_map(V, g.mods[m], mm);
        int32_t qb0, qb1;
        row_range(mm, knv, xl, xh, yl, yh, qb0, qb1);
        if (lds_cells)
            for (int32_t q = lane; q < cpm; q += 64) cc[q] = 0;
        __builtin_amdgcn_wave_barrier();
        for (int32_t qb = qb0; qb <= qb1; qb++) {
            const double fv = fv_tab[qb];
            int32_t qa0, qa1;
            col_range(mm, fv, knu, xl, xh, yl, yh, qa0, qa1);
            for (int32_t qa = qa0 + lane; qa <= qa1; qa += 64) {
                int32_t li, lj, zs;
                if (!sample_in_rect(mm, fu_tab[qa], fv, r, c.n, &li, &lj, &zs)) continue;
                const int32_t lx = li + r.x - c.x0, ly = lj + r.y - c.y0;
                if ((int64_t)zs > (int64_t)zt[ly * PITCH + lx] + (int64_t)bm) {
                    const int32_t cu = qa / k, cv = qb / k;
                    const int32_t cell = cv * g.n_cu + cu;
                    if (lds_cells) atomicAdd(&cc[cell], 1u);
                    else dev_add(&out.counts[(int64_t)m * cpm + cell], 1u);
                    if (out.bits) {
                        const int32_t si = (qb - cv * k) * k + (qa - cu * k);
                        dev_or(&out.bits[((int64_t)m * cpm + cell) * words + si / 32], 1u << (si % 32));
                    }
                }
            }
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
        if (lds_cells)
            for (int32_t q = lane; q < cpm; q += 64) {
                const uint32_t v = cc[q];
                if (v) dev_add(&out.counts[(int64_t)m * cpm + q], v);
            }
        __builtin_amdgcn_wave_barrier();
    }
}

// Sparse-route sample entry: texel (li, lj) in the rect, shading threshold
// (shaded iff threshold > nearest depth at the texel), and the sample's
// identity (tile module slot, qa, qb).
struct SparseLds {
    uint16_t* texel;     // lj * TS + li, and kShadedBit once a covering depth below thr is found
    int32_t* thr;        // zs - bias
    uint32_t* code;      // slot << 24 | qb << 12 | qa
    uint16_t* order;     // entries sorted by 8 x 8 stamp
};
// A sample is shaded when some covering depth lies below its threshold; only
// that flag is kept, in the top bit of its texel (texels of a tile of at most
// 128 x 128 need 14 bits).
constexpr uint16_t kShadedBit = 0x8000;
constexpr uint16_t kTexelMask = 0x3FFF;

struct SparseShared {
    int32_t n_ent, ent_overflow, max_thr, next, n_slots, cut;
    int32_t wsum[4];
};

// Light-space maps of the first kMapCache module slots of a tile are kept in
// LDS while its samples are listed.
constexpr int kMapCache = 64;

// A triangle of the current chunk, relative to the rect origin: edge k at
// texel (li, lj) of the rect is ex[k] + A[k] li + B[k] lj, depth
// (zx + gx li + gy lj) >> 16; box = clipped texel box (4 x 8 bits).
struct TriSlot {
    int64_t ex[3];          // edge values at the rect origin
    int32_t A[3], B[3];     // edge coefficients; a texel step adds 256 A (256 B)
    int64_t zx, gx, gy;
    uint32_t box, pad;
};

// A module's plane in light space, P(x, y) = z0 + a (x - x0) + b (y - y0) (x, y
// in texels, P in depth units), the plane its samples lie on, with the margin
// lim by which a slot's depth must exceed P for the slot to shade none of the
// module's samples. A sample s is tested at the centre c of its texel (|s - c|
// <= 1/2 in x and in y), so its depth z is at most P(c) + (|a| + |b|) / 2. A
// slot's depth there is floor(Q(c)) for its exact affine Q (clamped to [0,
// 2^24 - 1]: the clamp at 0 only raises it, and no sample depth exceeds the
// other end). The sample is lit, floor(z) - bias <= floor(Q(c)), whenever
// z - bias < Q(c), which holds when Q(c) - P(c) > (|a| + |b|) / 2 - bias + e,
// e the rounding of z and of P here. lim adds 0.01 plus a bound of that
// rounding; a bias at the cap leaves every sample lit. A module seen too nearly
// edge-on for a well-conditioned solve drops nothing (ok = false).
struct ModPlane {
    double x0, y0, z0, a, b, lim;
    bool ok, lit;
};

__device__ __forceinline__ ModPlane mod_plane(const ModMap& mm, int32_t bias, int32_t n) {
    ModPlane P;
    const double det = mm.du.x * mm.dv.y - mm.du.y * mm.dv.x;
    const double scale = (fabs(mm.du.x) + fabs(mm.du.y)) * (fabs(mm.dv.x) + fabs(mm.dv.y));
    P.a = (mm.du.z * mm.dv.y - mm.dv.z * mm.du.y) / det;
    P.b = (mm.dv.z * mm.du.x - mm.du.z * mm.dv.x) / det;
    P.x0 = mm.p0.x;
    P.y0 = mm.p0.y;
    P.z0 = mm.p0.z;
    const double big = fabs(mm.p0.z) + (fabs(P.a) + fabs(P.b)) * (2.0 * (double)n + fabs(mm.p0.x) + fabs(mm.p0.y));
    P.lim = 0.5 * (fabs(P.a) + fabs(P.b)) - (double)bias + 0.01 + 1e-9 * big;
    P.ok = fabs(det) >= 1e-5 * scale && isfinite(P.lim);
    P.lit = bias >= (int32_t)kDepthMax;
    return P;
}

// True when slot T shades no sample of the module: over the slot's texel box in
// the rect, where Q - P is smallest at a corner (both are affine), Q - P >= lim.
__device__ __forceinline__ bool slot_behind(const TriSlot& T, const ModPlane& P, const Rect& r) {
    if (P.lit) return true;
    if (!P.ok) return false;
    const uint32_t bx = T.box;
    double dmin = INFINITY;
    for (int q = 0; q < 4; q++) {
        const int32_t li = (q & 1) ? (int32_t)((bx >> 8) & 255u) : (int32_t)(bx & 255u);
        const int32_t lj = (q & 2) ? (int32_t)(bx >> 24) : (int32_t)((bx >> 16) & 255u);
        const double Q = (double)(T.zx + T.gx * li + T.gy * lj) / 65536.0;     // exact: below 2^53
        const double Pc = P.z0 + P.a * ((double)(r.x + li) + 0.5 - P.x0) + P.b * ((double)(r.y + lj) + 0.5 - P.y0);
        dmin = fmin(dmin, Q - Pc);
    }
    return dmin >= P.lim;
}

constexpr int kTriChunk = 64;     // triangles staged in LDS at a time
constexpr int kStampList = 48;    // triangle slots listed per 8x8 stamp (even: the test reads them in pairs)
static_assert(kStampList % 2 == 0, "stamp lists are read two bytes at a time");

struct TriBins {
    TriSlot* slot;      // [kTriChunk]
    int32_t* cnt;       // [64] triangles per stamp
    uint8_t* list;      // [64][kStampList]
};

// Sparse route over one rect of the tile: list the samples whose texel lies
// in the rect, test every binned triangle at their texel centres, count the
// shaded ones. Returns false (nothing written) when the rect holds more
// samples than the LDS list; the caller then splits it.
template <int TS, int CAP>
__device__ bool sparse_rect(const Rect& r, SparseLds& sp, SparseShared& sh, TriBins& tb, int32_t* rowstart, uint32_t* cells,
                            const int32_t* mods, int32_t n_mods, const View& V, const BinBuffers& bb, const GenDev& g,
                            const int32_t* bias, const double* fu_tab, const double* fv_tab, int32_t k,
                            const TileOut& out, const TileCtx& c, int tid, int lane, int wv) {
    const int32_t cpm = g.n_cu * g.n_cv;
    const int32_t knu = k * g.n_cu, knv = k * g.n_cv;
    double xl, xh, yl, yh;
    rect_bounds(r, c.n, xl, xh, yl, yh);
    if (tid == 0) { sh.n_ent = 0; sh.ent_overflow = 0; sh.max_thr = INT32_MIN; sh.next = 0; }
    for (int q = tid; q <= r.size; q += 256) rowstart[q] = 0;
    __syncthreads();
    // 1. the samples whose texel lies in the rect, in three steps: a thread per
    //    module finds its light-space map and conservative row range; a thread
    //    per row finds the row's column range; the (row, column) candidates are
    //    then spread evenly over all threads, each finding its row by binary
    //    search, and the entries are allocated once per wave. The fractions come
    //    from the sample tables (the same correctly rounded quotients
    //    (q + 1/2) / (k n)), in LDS when the workgroup holds a copy: one division
    //    per sample coordinate was part of what made listing half of the rooftop
    //    workload's tile time.
    //    Meanwhile `cells` holds the row tables, the triangle slots the map
    //    cache and the (not yet used) entry order the module biases.
    uint32_t* const mstart = cells;            // [256] (first row << 12) | first row index qb0, per module slot
    uint32_t* const rmq = cells + 256;         // [256] (module slot << 12) | qb, per row of a pass
    uint32_t* const ra0 = cells + 512;         // [256] first column of the row's range
    uint32_t* const rst = cells + 768;         // [256] first candidate of the row
    ModMap* const mcache = reinterpret_cast<ModMap*>(tb.slot);
    int32_t* const mbias = reinterpret_cast<int32_t*>(sp.order);
    static_assert(sizeof(ModMap) * kMapCache <= sizeof(TriSlot) * kTriChunk, "map cache exceeds the slot area");
    static_assert(kMaxTileMods <= 256 && 4 * kMaxTileMods <= 2 * CAP, "one thread per module slot, biases in the order area");
    int32_t my_max = INT32_MIN;
    int32_t n_rows;
    {
        int32_t rows = 0, qb0 = 0;
        if (tid < n_mods) {
            const int32_t m = mods[tid];
            const int32_t bm = bias[m];
            mbias[tid] = bm;
            if (bm >= 0) {                              // back-lit modules have no samples to test
                ModMap mm;
                module_map(V, g.mods[m], mm);
                if (tid < kMapCache) mcache[tid] = mm;
                int32_t qb1;
                row_range(mm, knv, xl, xh, yl, yh, qb0, qb1);
                rows = qb0 <= qb1 ? qb1 - qb0 + 1 : 0;
            }
        }
        const int32_t first = block_scan_excl(rows, sh.wsum, n_rows, lane, wv);
        if (tid < n_mods) mstart[tid] = ((uint32_t)first << 12) | (uint32_t)qb0;
        __syncthreads();
    }
    for (int32_t p0 = 0; p0 < n_rows; p0 += 256) {
        const int32_t rho = p0 + tid;
        int32_t cnt = 0;
        uint32_t rq = 0, a0 = 0;
        if (rho < n_rows) {
            const int32_t mi = last_at_most<12>(mstart, n_mods, (uint32_t)rho);
            const int32_t qb = (int32_t)(mstart[mi] & 0xFFFu) + rho - (int32_t)(mstart[mi] >> 12);
            ModMap mm;
            if (mi < kMapCache) mm = mcache[mi];
            else module_map(V, g.mods[mods[mi]], mm);
            const double fv = frac_v(c, qb);                 // the sample's fraction along edge_v
            int32_t qa0, qa1;
            col_range(mm, fv, knu, xl, xh, yl, yh, qa0, qa1);
            cnt = qa0 <= qa1 ? qa1 - qa0 + 1 : 0;
            rq = ((uint32_t)mi << 12) | (uint32_t)qb;
            a0 = (uint32_t)qa0;
        }
        int32_t n_cand;
        const int32_t first = block_scan_excl(cnt, sh.wsum, n_cand, lane, wv);
        rmq[tid] = rq;
        ra0[tid] = a0;
        rst[tid] = (uint32_t)first;
        __syncthreads();
        const int32_t nr = min(256, n_rows - p0);
        for (int32_t c0 = 0; c0 < n_cand; c0 += 256) {
            const int32_t cand = c0 + tid;
            bool ok = false;
            int32_t li = 0, lj = 0, th = 0;
            uint32_t code = 0;
            if (cand < n_cand) {
                const int32_t row = last_at_most<0>(rst, nr, (uint32_t)cand);
                const uint32_t q = rmq[row];
                const int32_t mi = (int32_t)(q >> 12), qb = (int32_t)(q & 0xFFFu);
                const int32_t qa = (int32_t)ra0[row] + cand - (int32_t)rst[row];
                ModMap mm;
                const int32_t bm = mbias[mi];
                if (mi < kMapCache) mm = mcache[mi];
                else module_map(V, g.mods[mods[mi]], mm);
                const double fv = frac_v(c, qb);
                const double fu = frac_u(c, qa);                 // the sample's fraction along edge_u
                int32_t zs;
                ok = sample_in_rect(mm, fu, fv, r, c.n, &li, &lj, &zs);
                if (ok) {
                    const int64_t th64 = (int64_t)zs - (int64_t)bm;
                    th = th64 < (int64_t)INT32_MIN ? INT32_MIN : (int32_t)th64;
                    code = ((uint32_t)mi << 24) | ((uint32_t)qb << 12) | (uint32_t)qa;
                    my_max = max(my_max, th);
                }
            }
            const unsigned long long bal = __ballot(ok);
            int32_t wbase = 0;
            if (lane == 0 && bal) wbase = atomicAdd(&sh.n_ent, __popcll(bal));
            wbase = __builtin_amdgcn_readfirstlane(wbase);
            if (ok) {
                const int32_t e = wbase + lanes_below(bal);
                if (e >= CAP) {
                    sh.ent_overflow = 1;
                } else {
                    sp.texel[e] = (uint16_t)(lj * TS + li);
                    sp.thr[e] = th;
                    sp.code[e] = code;
                }
            }
        }
        __syncthreads();                                   // the row tables are rewritten by the next pass
    }
    for (int off = 1; off < 64; off <<= 1) my_max = max(my_max, __shfl_xor(my_max, off, 64));
    if (lane == 0 && my_max != INT32_MIN) atomicMax(&sh.max_thr, my_max);
    __syncthreads();
    if (sh.ent_overflow) return false;
    const int32_t ne = sh.n_ent;
    if (ne == 0) return true;
    // 2. counting sort of the entries by 8x8 stamp of the rect
    const int32_t spr = (r.size + 7) / 8, n_st = spr * spr;
    for (int32_t e = tid; e < ne; e += 256) {
        const int32_t tx = sp.texel[e] & kTexelMask;
        atomicAdd(&rowstart[(tx / TS / 8) * spr + (tx % TS) / 8 + 1], 1);
    }
    __syncthreads();
    if (wv == 0) {                                  // inclusive scan of the <= 64 stamp counts
        int32_t x = lane < n_st ? rowstart[lane + 1] : 0;
        for (int off = 1; off < 64; off <<= 1) {
            const int32_t y = __shfl_up(x, off, 64);
            if (lane >= off) x += y;
        }
        if (lane < n_st) rowstart[lane + 1] = x;
    }
    __syncthreads();
    for (int q = tid; q < n_st; q += 256) cells[q] = (uint32_t)rowstart[q];
    __syncthreads();
    for (int32_t e = tid; e < ne; e += 256) {
        const int32_t tx = sp.texel[e] & kTexelMask;
        sp.order[atomicAdd(&cells[(tx / TS / 8) * spr + (tx % TS) / 8], 1u)] = (uint16_t)e;
    }
    // 3. triangles in chunks of up to kTriChunk: the records that reach the
    //    rect go to LDS (relative to the rect origin), are binned into the
    //    rect's stamps one lane per stamp, and every sample then tests only
    //    the triangles of its own stamp. A chunk is filled 256 candidates at
    //    a time: every thread tests one, the survivors take the free slots in
    //    candidate order, and the walk goes on after the last one placed, so
    //    a rect that few of its tile's triangles reach (a quadrant item) takes
    //    few chunks.
    const int32_t mthr = sh.max_thr;
    const int32_t total = c.n_large + (c.be - c.bs);
    int32_t base = 0;
    while (base < total) {
        for (int q = tid; q < n_st; q += 256) tb.cnt[q] = 0;
        int32_t ns = 0;
        while (ns < kTriChunk && base < total) {      // uniform: base and ns follow block totals
            const int32_t item = base + tid;
            bool keep = false;
            TriRec R;
            TriClip t;
            if (item < total) {
                bool have = item < c.n_lrec;
                if (have) {
                    R = c.lrec[item];
                } else {
                    const int32_t rid = item < c.n_large ? bb.large[item] : bb.bins[c.bs + item - c.n_large];
                    if (rid >= 0) {
                        R = bb.rec[rid];
                        have = true;
                    }
                }
                if (have) {
                    if (clip_to_rect(R, r, t)) {
                        const int64_t zmin = R.z0 + R.gx * (R.gx > 0 ? t.ilo : t.ihi) + R.gy * (R.gy > 0 ? t.jlo : t.jhi);
                        keep = (int64_t)depth_q(zmin) < (int64_t)mthr;
                    }
                }
            }
            int32_t n_keep;
            const int32_t rank = block_scan_excl(keep ? 1 : 0, sh.wsum, n_keep, lane, wv);
            const int32_t room = kTriChunk - ns;
            if (keep && rank < room) {
                TriSlot& T = tb.slot[ns + rank];
                for (int e = 0; e < 3; e++) {
                    T.ex[e] = edge_at(R.e0[e], R.a[e], R.b[e], 256 * r.x, 256 * r.y);
                    T.A[e] = R.a[e];
                    T.B[e] = R.b[e];
                }
                T.zx = R.z0 + R.gx * r.x + R.gy * r.y;
                T.gx = R.gx;
                T.gy = R.gy;
                T.box = (uint32_t)(t.ilo - r.x) | ((uint32_t)(t.ihi - r.x) << 8) | ((uint32_t)(t.jlo - r.y) << 16) |
                        ((uint32_t)(t.jhi - r.y) << 24);
            }
            if (keep && rank == room) sh.cut = tid;        // the first survivor left for the next chunk
            if (n_keep > room) {
                __syncthreads();
                base += sh.cut;
                ns = kTriChunk;
            } else {
                base += 256;
                ns += n_keep;
            }
        }
        __syncthreads();
        if (ns == 0) break;
        // stamp binning: wave per triangle slot, lane per stamp
        for (int32_t q = wv; q < ns; q += 4) {
            const TriSlot& T = tb.slot[q];
            const int32_t bi0 = (int32_t)(T.box & 255), bi1 = (int32_t)((T.box >> 8) & 255);
            const int32_t bj0 = (int32_t)((T.box >> 16) & 255), bj1 = (int32_t)(T.box >> 24);
            if (lane < n_st) {
                const int32_t sx = (lane % spr) * 8, sy = (lane / spr) * 8;
                const int32_t i0 = max(sx, bi0), i1 = min(sx + 7, bi1), j0 = max(sy, bj0), j1 = min(sy + 7, bj1);
                bool hit = i0 <= i1 && j0 <= j1;
                for (int e = 0; e < 3 && hit; e++) {
                    const int64_t emax = edge_at(T.ex[e], T.A[e], T.B[e], 256 * (T.A[e] > 0 ? i1 : i0),
                                                 256 * (T.B[e] > 0 ? j1 : j0));
                    hit = emax >= 0;
                }
                if (hit) {
                    const int32_t pos = atomicAdd(&tb.cnt[lane], 1);
                    if (pos < kStampList) tb.list[lane * kStampList + pos] = (uint8_t)q;
                }
            }
        }
        __syncthreads();
        // samples against the triangles of their stamp (all triangles of the chunk when the list overflowed)
        for (int32_t p = tid; p < ne; p += 256) {
            const int32_t e = sp.order[p];
            const uint16_t tw = sp.texel[e];
            if (tw & kShadedBit) continue;                  // settled by an earlier chunk
            const int32_t tx = tw & kTexelMask;
            const int32_t li = tx % TS, lj = tx / TS;
            const int32_t li256 = li * 256, lj256 = lj * 256;
            const int32_t st = (lj / 8) * spr + li / 8;
            const int32_t nl = tb.cnt[st];
            const bool all = nl > kStampList;
            const int32_t nt = all ? ns : nl;
            // only whether the sample is shaded is kept, and a covering depth
            // below its threshold settles that: the search stops there. The
            // triangles go two at a time (their list bytes read together, both
            // slot reads in flight at once); testing the second after the first
            // has hit changes nothing (C2 year 328 -> 322 ms)
            const int32_t thr = sp.thr[e];
            bool shaded = false;
            for (int32_t u0 = 0; u0 < nt; u0 += 2) {
                const uint32_t qp = all ? ((uint32_t)u0 | ((uint32_t)(u0 + 1) << 8))
                                        : (uint32_t)*reinterpret_cast<const uint16_t*>(&tb.list[st * kStampList + u0]);
                bool hit = false;
#pragma unroll
                for (int v = 0; v < 2; v++) {
                    if (u0 + v < nt) {
                        const TriSlot& T = tb.slot[(qp >> (8 * v)) & 255u];
                        const int64_t E0 = edge_at(T.ex[0], T.A[0], T.B[0], li256, lj256);
                        const int64_t E1 = edge_at(T.ex[1], T.A[1], T.B[1], li256, lj256);
                        const int64_t E2 = edge_at(T.ex[2], T.A[2], T.B[2], li256, lj256);
                        hit |= (E0 | E1 | E2) >= 0 && thr > (int32_t)depth_q(T.zx + T.gx * li + T.gy * lj);
                    }
                }
                if (hit) {
                    shaded = true;
                    break;
                }
            }
            if (shaded) sp.texel[e] = tw | kShadedBit;
        }
        __syncthreads();
    }
    __syncthreads();
    // 4. shaded flags, per-cell counts
    const bool lds_cells = n_mods * cpm <= kMaxTileCells;
    if (lds_cells)
        for (int32_t q = tid; q < n_mods * cpm; q += 256) cells[q] = 0;
    __syncthreads();
    const int32_t words = (k * k + 31) / 32;
    const DivK dk = div_by(k);
    const int32_t n_cu = g.n_cu;
    for (int32_t e = tid; e < ne; e += 256) {
        if (!(sp.texel[e] & kShadedBit)) continue;
        const uint32_t code = sp.code[e];
        const int32_t slot = (int32_t)(code >> 24), qb = (int32_t)((code >> 12) & 0xFFF), qa = (int32_t)(code & 0xFFF);
        const int32_t cu = div_k(dk, qa), cv = div_k(dk, qb), cell = cv * n_cu + cu;
        const int32_t m = mods[slot];
        if (lds_cells) atomicAdd(&cells[slot * cpm + cell], 1u);
        else dev_add(&out.counts[(int64_t)m * cpm + cell], 1u);
        if (out.bits) {
            const int32_t si = (qb - cv * k) * k + (qa - cu * k);
            dev_or(&out.bits[((int64_t)m * cpm + cell) * words + si / 32], 1u << (si % 32));
        }
    }
    __syncthreads();
    if (lds_cells)
        for (int32_t q = tid; q < n_mods * cpm; q += 256) {
            const uint32_t v = cells[q];
            if (v) dev_add(&out.counts[(int64_t)mods[q / cpm] * cpm + q % cpm], v);
        }
    __syncthreads();
    return true;
}

constexpr int kMinRect = 16;
constexpr int kMaxRects = 64;

// Sample entries a rect of the sparse route may hold (a denser rect is split
// in four): 12 bytes each, sized so that 64-texel tiles of the row-plant
// workload (up to about 2,450 samples) never split.
constexpr int kCap32 = 1364, kCap64 = 2730, kCap128 = 5460;

template <int TS, int CAP>
struct TileLds {
    static constexpr int PITCH = TS + 8;
    static constexpr int ZT_BYTES = TS * PITCH * 4;
    static constexpr int SP_BYTES = CAP * (2 + 4 + 4 + 2);
    static_assert(CAP % 2 == 0 && TS <= 128, "aligned entry arrays; texels below kShadedBit");
    static constexpr int POOL = ZT_BYTES > SP_BYTES ? ZT_BYTES : SP_BYTES;
    __attribute__((aligned(16))) unsigned char pool[POOL];
    int32_t mods[kMaxTileMods];
    uint32_t cells[kMaxTileCells > 4 * kMaxCellCounters ? kMaxTileCells : 4 * kMaxCellCounters];
    int32_t rowstart[TS + 1];
    Rect todo[kMaxRects], failed[kMaxRects];
    TriSlot tslots[kTriChunk];
    int32_t tcnt[64];
    alignas(4) uint8_t tlist[64 * kStampList];   // read two bytes at a time
    int32_t next, n_mods, mods_overflow, n_todo, n_failed;
    SparseShared sh;
    TriRec lcache[kLargeCache];
    double ftab[kFracCache];
    static_assert(TS != 64 || 4 * kWaveSlots * sizeof(TriSlot) <= POOL, "wave slots of four waves fit the pool");
};

// One work item of one sun: a tile, or a quadrant of it (the tile's samples
// in that quadrant, against every triangle binned to the tile). V, bias_s and
// n_large are this sun's view, module biases and count of unbinned triangles.
template <int TS, int CAP>
__device__ __attribute__((always_inline)) void tile_body(TileLds<TS, CAP>& L, int32_t item, int32_t n_lcache, bool lds_tables, const View& V, const BinBuffers& bb, int32_t n_large,
                          int32_t n, const GenDev& g, const int32_t* bias, const double* fu_tab,
                          const double* fv_tab, int32_t k, const TileOut& out, int32_t sparse,
                          const uint32_t* tmask) {
    constexpr int PITCH = TS + 8;
    auto& pool = L.pool;
    auto& mods = L.mods;
    auto& cells = L.cells;
    auto& rowstart = L.rowstart;
    auto& todo = L.todo;
    auto& failed = L.failed;
    auto& tslots = L.tslots;
    auto& tcnt = L.tcnt;
    auto& tlist = L.tlist;
    auto& next = L.next;
    auto& n_mods = L.n_mods;
    auto& mods_overflow = L.mods_overflow;
    auto& n_todo = L.n_todo;
    auto& n_failed = L.n_failed;
    auto& sh = L.sh;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int32_t tile = item >> 3, part = item & 7;
    TileCtx c;
    c.n = n;
    c.x0 = (tile % bb.ntx) * TS;
    c.y0 = (tile / bb.ntx) * TS;
    uint32_t* zt = reinterpret_cast<uint32_t*>(pool);
    if (V.valid && !out.map && !mask_has(tmask, tile)) return;   // no sample can fall in this tile
    if (!V.valid) {
        if (out.map) {                            // nothing drawn: the exported picture stays at the far depth
            for (int q = tid; q < TS * TS; q += 256) {
                const int32_t py = c.y0 + q / TS, px = c.x0 + q % TS;
                if (py < n && px < n) out.map[(int64_t)py * n + px] = kDepthMax;
            }
        }
        return;
    }
    c.bs = min(bb.tile_start[tile], bb.bin_cap);
    c.be = min(bb.tile_start[tile + 1], bb.bin_cap);
    c.n_large = n_large;
    c.lrec = L.lcache;
    c.n_lrec = n_lcache;
    c.ftab = L.ftab;
    c.fu_g = fu_tab;
    c.fv_g = fv_tab;
    c.knu = k * g.n_cu;
    c.lds = lds_tables;
    if (tid == 0) { next = 0; n_mods = 0; mods_overflow = 0; n_todo = 0; n_failed = 0; }
    __syncthreads();
    for (int32_t q = c.bs + tid; q < c.be; q += 256) {   // module entries of this tile
        const int32_t id = bb.bins[q];
        if (id < 0) {
            const int32_t slot = atomicAdd(&n_mods, 1);
            if (slot < kMaxTileMods) mods[slot] = -id - 1;
            else mods_overflow = 1;
        }
    }
    __syncthreads();
    const bool test = out.test && n_mods > 0;
    if (!test && !out.map) return;                        // no sample falls here and nothing to export
    const Rect whole{c.x0, c.y0, TS};

    if (sparse && !out.map && test && !mods_overflow) {
        SparseLds sp;
        sp.texel = reinterpret_cast<uint16_t*>(pool);
        sp.thr = reinterpret_cast<int32_t*>(pool + 2 * CAP);
        sp.code = reinterpret_cast<uint32_t*>(pool + 6 * CAP);
        sp.order = reinterpret_cast<uint16_t*>(pool + 10 * CAP);
        TriBins tb;
        tb.slot = tslots;
        tb.cnt = tcnt;
        tb.list = tlist;
        // Nothing to count when every triangle that reaches the item's rect lies far enough behind the
        // plane of every module here (its own triangles, a roof under it; see ModPlane), over the
        // triangle's box in the rect: settled before any sample is listed. A sub-rect of a later split
        // holds a part of each box, where the bound still holds.
        {
            const int32_t h = TS / 2;
            const Rect er = part == kWholeTile ? whole : Rect{c.x0 + (part & 1) * h, c.y0 + (part >> 1) * h, h};
            ModPlane* const planes = reinterpret_cast<ModPlane*>(pool);
            static_assert(sizeof(ModPlane) * kMaxTileMods <= sizeof(pool), "a plane per module slot in the pool");
            if (tid < n_mods) {
                const int32_t m = mods[tid];
                const int32_t bm = bias[m];
                ModPlane mp{};
                mp.lit = true;                            // back-lit: none of its samples is tested
                if (bm >= 0) {
                    ModMap mm;
                    module_map(V, g.mods[m], mm);
                    mp = mod_plane(mm, bm, n);
                }
                planes[tid] = mp;
            }
            __syncthreads();
            const int32_t total = c.n_large + (c.be - c.bs);
            bool front = false;
            for (int32_t b0 = 0; b0 < total && !front; b0 += 256) {
                const int32_t it = b0 + tid;
                bool fr = false;
                if (it < total) {
                    TriRec R;
                    bool have = it < c.n_lrec;
                    if (have) {
                        R = c.lrec[it];
                    } else {
                        const int32_t rid = it < c.n_large ? bb.large[it] : bb.bins[c.bs + it - c.n_large];
                        if (rid >= 0) {
                            R = bb.rec[rid];
                            have = true;
                        }
                    }
                    TriClip t;
                    if (have && clip_to_rect(R, er, t)) {
                        TriSlot T;
                        T.zx = R.z0 + R.gx * er.x + R.gy * er.y;
                        T.gx = R.gx;
                        T.gy = R.gy;
                        T.box = (uint32_t)(t.ilo - er.x) | ((uint32_t)(t.ihi - er.x) << 8) |
                                ((uint32_t)(t.jlo - er.y) << 16) | ((uint32_t)(t.jhi - er.y) << 24);
                        for (int32_t mi = 0; mi < n_mods && !fr; mi++) fr = !slot_behind(T, planes[mi], er);
                    }
                }
                front = __syncthreads_or(fr) != 0;
            }
            if (!front) return;
            __syncthreads();                              // the pool takes the sample lists next
        }
        if (tid == 0) {                               // rects of at most 64 x 64 texels (one lane per 8x8 stamp)
            n_todo = 0;
            if (part != kWholeTile) {
                const int32_t h = TS / 2;
                todo[n_todo++] = Rect{c.x0 + (part & 1) * h, c.y0 + (part >> 1) * h, h};
            } else {
                const int32_t rs = TS < 64 ? TS : 64;
                for (int32_t y = 0; y < TS; y += rs)
                    for (int32_t x = 0; x < TS; x += rs) todo[n_todo++] = Rect{c.x0 + x, c.y0 + y, rs};
            }
        }
        __syncthreads();
        while (n_todo > 0) {                              // a rect with too many samples is split in four
            const Rect r = todo[n_todo - 1];
            __syncthreads();
            if (tid == 0) n_todo--;
            const bool ok = sparse_rect<TS, CAP>(r, sp, sh, tb, rowstart, cells, mods, n_mods, V, bb, g, bias, fu_tab,
                                                 fv_tab, k, out, c, tid, lane, wv);
            if (tid == 0 && !ok) {
                if (r.size > kMinRect && n_todo + 4 <= kMaxRects) {
                    const int32_t h = r.size / 2;
                    todo[n_todo++] = Rect{r.x, r.y, h};
                    todo[n_todo++] = Rect{r.x + h, r.y, h};
                    todo[n_todo++] = Rect{r.x, r.y + h, h};
                    todo[n_todo++] = Rect{r.x + h, r.y + h, h};
                } else if (n_failed < kMaxRects) {
                    failed[n_failed++] = r;
                }
            }
            __syncthreads();
        }
        if (n_failed == 0) return;
        if (tid == 0) next = 0;                           // full route for the rects that stayed too dense
        __syncthreads();
    } else {
        if (tid == 0) {
            const int32_t h = TS / 2;
            failed[0] = part == kWholeTile ? whole : Rect{c.x0 + (part & 1) * h, c.y0 + (part >> 1) * h, h};
            n_failed = 1;
        }
        __syncthreads();
    }

    // full route
    for (int q = tid; q < TS * PITCH; q += 256) zt[q] = kDepthMax;
    __syncthreads();
    raster_full<TS>(zt, &next, bb, c, lane);
    __syncthreads();
    if (out.map) store_tile<TS>(zt, out.map, c, tid);
    if (!test) return;
    const int32_t nm = mods_overflow ? (c.be - c.bs) : n_mods;
    for (int32_t f = 0; f < n_failed; f++)
        samples_full<TS>(zt, mods, nm, !mods_overflow, cells + wv * kMaxCellCounters, V, bb, g, bias, fu_tab, fv_tab,
                         k, out, c, failed[f], lane, wv);
}

// ---------------------------------------------------------------------------
// Light tiles, one wave each. A tile with few bin entries (its modules and a
// few triangles) and a short large list is evaluated by a single wave with no
// workgroup barrier and no sample list: the wave stages the tile's triangles
// that can shade a sample in its own LDS slots, then its lanes take the
// tile's samples straight from each module's row and column ranges and test
// each against every staged triangle. The samples, the triangles tested and
// the test itself are those of the workgroup route, so every count is the
// same; only the order of the work differs.
// ---------------------------------------------------------------------------

// DPP control of a move from lane i - 1 to lane i across the whole wave (wave_shr:1).
constexpr int kDppWaveShr1 = 0x138;

// Inclusive prefix sum over the lanes of a wave.
__device__ __forceinline__ int32_t wave_incl(int32_t x, int lane) {
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

// The number of lanes whose (non-decreasing) incl is at most x, at most 63.
__device__ __forceinline__ int32_t wave_count_le(int32_t incl, int32_t x) {
    int32_t lo = 0;
    for (int step = 32; step >= 1; step >>= 1) {
        const int32_t v = __shfl(incl, lo + step - 1, 64);
        if (v <= x) lo += step;
    }
    return lo;
}

__device__ __forceinline__ int32_t wave_max(int32_t v) {
    for (int off = 1; off < 64; off <<= 1) v = max(v, __shfl_xor(v, off, 64));
    return v;
}

template <int TS>
__device__ void wave_tile(TriSlot* slots, int32_t tile, const View& V, const BinBuffers& bb,
                          int32_t n_large, int32_t n, const GenDev& g, const int32_t* bias, const double* fu_l,
                          const double* fv_l, int32_t k, const TileOut& out, int lane) {
    // a listed tile holds bin entries, which only tiles of the tile mask get
    if (!V.valid) return;
    const Rect r{(tile % bb.ntx) * TS, (tile / bb.ntx) * TS, TS};
    const int32_t bs = min(bb.tile_start[tile], bb.bin_cap), be = min(bb.tile_start[tile + 1], bb.bin_cap);
    const int32_t ne = be - bs;                            // below 8 kLightBuckets: one entry per lane
    const int32_t id = lane < ne ? bb.bins[bs + lane] : 0;
    const bool is_mod = lane < ne && id < 0;
    const unsigned long long mb = __ballot(is_mod);
    if (mb == 0ull) return;                                // no module here: nothing to test
    // an upper bound of the samples' thresholds: the module's farthest corner, floored,
    // plus two, less its bias (a sample lies inside its module's corners)
    // (the corners are read whatever the bias, so both loads are in flight together; a module
    // lane keeps its bias for the module loops below)
    int32_t bound = INT32_MIN, bias_l = -1;
    if (is_mod) {
        const int32_t m = -id - 1;
        double zmax = -INFINITY;
        for (int q = 0; q < 4; q++) {
            d3 p;
            module_corner(g.mods[m], q, p);
            zmax = fmax(zmax, to_light(V, p).z);
        }
        bias_l = bias[m];
        if (bias_l >= 0) {
            const double b = floor(zmax) + 2.0 - (double)bias_l;
            bound = b >= 2147483647.0 ? INT32_MAX : (b <= -2147483648.0 ? INT32_MIN : (int32_t)b);
        }
    }
    const int32_t mthr = wave_max(bound);
    if (mthr == INT32_MIN) return;                         // every module here is back-lit
    // the triangles that reach the tile in front of some sample, in this wave's slots
    int32_t ns = 0;
    const int32_t n_cand = n_large + ne;                   // n_large <= kLargeCache: all in LDS
    for (int32_t c0 = 0; c0 < n_cand; c0 += 64) {
        const int32_t ci = c0 + lane;
        const int32_t rid = __shfl(id, (ci - n_large) & 63, 64);   // every lane takes part in the shuffle
        bool keep = false;
        TriRec R;
        TriClip t;
        if (ci < n_large) {
            R = bb.rec[bb.large[ci]];
            keep = true;
        } else if (ci < n_cand && rid >= 0) {
            R = bb.rec[rid];
            keep = true;
        }
        if (keep) {
            keep = clip_to_rect(R, r, t);
            if (keep) {
                const int64_t zmin = R.z0 + R.gx * (R.gx > 0 ? t.ilo : t.ihi) + R.gy * (R.gy > 0 ? t.jlo : t.jhi);
                keep = (int64_t)depth_q(zmin) < (int64_t)mthr;
            }
        }
        const unsigned long long kb = __ballot(keep);
        if (keep) {
            TriSlot& T = slots[ns + lanes_below(kb)];
            for (int e = 0; e < 3; e++) {
                T.ex[e] = edge_at(R.e0[e], R.a[e], R.b[e], 256 * r.x, 256 * r.y);
                T.A[e] = R.a[e];
                T.B[e] = R.b[e];
            }
            T.zx = R.z0 + R.gx * r.x + R.gy * r.y;
            T.gx = R.gx;
            T.gy = R.gy;
            T.box = (uint32_t)(t.ilo - r.x) | ((uint32_t)(t.ihi - r.x) << 8) | ((uint32_t)(t.jlo - r.y) << 16) |
                    ((uint32_t)(t.jhi - r.y) << 24);
        }
        ns += __popcll(kb);
    }
    if (ns == 0) return;                                   // nothing can shade a sample here
    // nothing either when every staged slot lies behind the plane of every module tested here (its
    // own triangles, a roof under it; see ModPlane): the common case, settled before the stamp masks.
    // Each module lane tests its own module's plane against every slot (the slot reads are the same
    // address on every lane), so the modules' terms are read and solved side by side.
    {
        bool front = false;
        if (is_mod && bias_l >= 0) {
            ModMap mm;
            module_map(V, g.mods[-id - 1], mm);
            const ModPlane mp = mod_plane(mm, bias_l, n);
            for (int32_t u = 0; u < ns && !front; u++) front = !slot_behind(slots[u], mp, r);
        }
        if (__ballot(front) == 0ull) return;
    }
    // lane s holds the slots that reach 8 x 8 stamp s of the tile (the stamp's box
    // against the triangle's box, then each edge at the stamp corner farthest inside)
    static_assert(TS == 64 && kWaveSlots <= 128, "a lane per stamp, two mask words");
    unsigned long long sm0 = 0ull, sm1 = 0ull;
    {
        const int32_t sx = (lane & 7) * 8, sy = (lane >> 3) * 8;
        for (int32_t u = 0; u < ns; u++) {
            const TriSlot& T = slots[u];
            const uint32_t bx = T.box;
            const int32_t i0 = max(sx, (int32_t)(bx & 255)), i1 = min(sx + 7, (int32_t)((bx >> 8) & 255));
            const int32_t j0 = max(sy, (int32_t)((bx >> 16) & 255)), j1 = min(sy + 7, (int32_t)(bx >> 24));
            bool hit = i0 <= i1 && j0 <= j1;
            for (int e = 0; e < 3 && hit; e++) {
                const int64_t emax = edge_at(T.ex[e], T.A[e], T.B[e], 256 * (T.A[e] > 0 ? i1 : i0),
                                             256 * (T.B[e] > 0 ? j1 : j0));
                hit = emax >= 0;
            }
            if (hit) {
                if (u < 64) sm0 |= 1ull << u;
                else sm1 |= 1ull << (u - 64);
            }
        }
    }
    // the samples of each module, 64 at a time (fields read once: stores through the output
    // pointers may alias them as far as the compiler knows)
    const int32_t n_cu = g.n_cu;
    const int32_t cpm = n_cu * g.n_cv;
    const int32_t knu = k * n_cu, knv = k * g.n_cv;
    const int32_t words = (k * k + 31) / 32;
    const DivK dk = div_by(k);
    uint32_t* const counts = out.counts;
    uint32_t* const bits = out.bits;
    double xl, xh, yl, yh;
    rect_bounds(r, n, xl, xh, yl, yh);
    unsigned long long todo = mb;
    while (todo) {
        const int src = __ffsll((long long)todo) - 1;
        todo &= todo - 1;
        const int32_t m = -__shfl(id, src, 64) - 1;
        const int32_t bm = __shfl(bias_l, src, 64);
        if (bm < 0) continue;                              // back-lit: not tested
        ModMap mm;
        module_map(V, g.mods[m], mm);
        int32_t qb0, qb1;
        row_range(mm, knv, xl, xh, yl, yh, qb0, qb1);
        // the slots that lie far enough behind the module's plane over their box to shade none of its
        // samples (its own triangles, a roof under it): its samples leave them out
        const ModPlane mp = mod_plane(mm, bm, n);
        const unsigned long long own0 = __ballot(lane < ns && slot_behind(slots[lane], mp, r));
        const unsigned long long own1 = __ballot(lane + 64 < ns && slot_behind(slots[lane + 64], mp, r));
        const unsigned long long any0 = __ballot(lane < ns), any1 = __ballot(lane + 64 < ns);
        if (((any0 & ~own0) | (any1 & ~own1)) == 0ull) continue;   // nothing left can shade its samples
        for (int32_t rb = qb0; rb <= qb1; rb += 64) {
            const int32_t qb_l = rb + lane;
            int32_t qa0 = 0, cnt = 0;
            if (qb_l <= qb1) {
                int32_t qa1;
                col_range(mm, fv_l[qb_l], knu, xl, xh, yl, yh, qa0, qa1);
                cnt = qa0 <= qa1 ? qa1 - qa0 + 1 : 0;
            }
            const int32_t incl = wave_incl(cnt, lane);
            const int32_t total = __builtin_amdgcn_readlane(incl, 63);
            for (int32_t c0 = 0; c0 < total; c0 += 64) {
                const int32_t ci = c0 + lane;
                const int32_t row = wave_count_le(incl, ci);
                const int32_t before = __shfl(incl - cnt, row, 64);
                const int32_t qa = __shfl(qa0, row, 64) + (ci - before);
                const int32_t qb = rb + row;
                bool live = false;
                int32_t li = 0, lj = 0, thr = 0;
                if (ci < total) {
                    int32_t zs;
                    live = sample_in_rect(mm, fu_l[qa], fv_l[qb], r, n, &li, &lj, &zs);
                    const int64_t th64 = (int64_t)zs - (int64_t)bm;
                    thr = th64 < (int64_t)INT32_MIN ? INT32_MIN : (int32_t)th64;
                }
                // the slots of the sample's stamp (every lane takes part in the shuffles)
                const int32_t st = (lj >> 3) * 8 + (li >> 3);
                unsigned long long m0 = __shfl(sm0, st, 64) & ~own0, m1 = __shfl(sm1, st, 64) & ~own1;
                if (!live) m0 = m1 = 0ull;
                bool shaded = false;
                const int32_t li256 = li * 256, lj256 = lj * 256;
                while ((m0 | m1) != 0ull && !shaded) {
                    int32_t u;
                    if (m0) {
                        u = __ffsll((long long)m0) - 1;
                        m0 &= m0 - 1;
                    } else {
                        u = 64 + __ffsll((long long)m1) - 1;
                        m1 &= m1 - 1;
                    }
                    const TriSlot& T = slots[u];
                    const int64_t E0 = edge_at(T.ex[0], T.A[0], T.B[0], li256, lj256);
                    const int64_t E1 = edge_at(T.ex[1], T.A[1], T.B[1], li256, lj256);
                    const int64_t E2 = edge_at(T.ex[2], T.A[2], T.B[2], li256, lj256);
                    shaded = (E0 | E1 | E2) >= 0 && thr > (int32_t)depth_q(T.zx + T.gx * li + T.gy * lj);
                }
                // the candidates of one cell lie on consecutive lanes (up to k of a row): the first
                // lane of each such run adds the run's shaded samples in one atomic
                const int32_t cu = div_k(dk, qa), cv = div_k(dk, qb);
                const int32_t key = live ? cv * n_cu + cu : -1 - lane;
                const int32_t below = __builtin_amdgcn_update_dpp(0, key, kDppWaveShr1, 0xf, 0xf, false);   // lane - 1's key
                const bool head = lane == 0 || key != below;
                const unsigned long long heads = __ballot(head), shaded_lanes = __ballot(shaded);
                if (head && live) {
                    const unsigned long long above = lane == 63 ? 0ull : (heads >> (lane + 1)) << (lane + 1);
                    const unsigned long long run = (above & (~above + 1ull)) - (1ull << lane);   // lanes [lane, next head)
                    const uint32_t n_shaded = (uint32_t)__popcll(shaded_lanes & run);
                    if (n_shaded) dev_add(&counts[(int64_t)m * cpm + key], n_shaded);
                }
                if (shaded && bits) {
                    const int32_t si = (qb - cv * k) * k + (qa - cu * k);
                    dev_or(&bits[((int64_t)m * cpm + key) * words + si / 32], 1u << (si % 32));
                }
            }
        }
    }
}

// Group form. With work lists (sparse route) the resident grid takes the suns
// in order, each sun's heaviest items first, so the light items at the end
// of one sun's list run beside the heavy ones at the start of the next;
// otherwise one workgroup per (tile, sun).
template <int TS, int CAP>
__global__ __launch_bounds__(256, 3) void k_tile_g(const SunGroup* __restrict__ grp, const View* views,
                                                const SunCounters* ctr, int32_t n, const int32_t* bias,
                                                const double* fu_tab, const double* fv_tab, int32_t k) {
    __shared__ TileLds<TS, CAP> L;
    __shared__ int32_t take;
    if (!grp->sun[0].bb.tile_list) {
        const GroupSun& S = grp->sun[blockIdx.y];
        tile_body<TS, CAP>(L, ((int32_t)blockIdx.x << 3) | kWholeTile, 0, false, views[S.s], S.bb, ctr[S.s].n_large, n, S.g,
                           bias + S.s * S.g.n_mod, fu_tab, fv_tab, k, S.out, S.out.sparse, S.tmask);
        return;
    }
    const int32_t ng = grp->n;
    // the sample fractions are the same for every sun of the evaluation
    const int32_t knu = k * grp->sun[0].g.n_cu, knv = k * grp->sun[0].g.n_cv;
    const bool lds_tables = knu + knv <= kFracCache;
    if (lds_tables)
        for (int32_t u = threadIdx.x; u < knu + knv; u += 256) L.ftab[u] = u < knu ? fu_tab[u] : fv_tab[u - knu];
    // The heavy items of every sun first, a workgroup each; then the light tiles of every sun, a
    // wave each, with no barrier between suns: the light route reads the sun's large triangles
    // from memory, so nothing in LDS changes with the sun. Each workgroup starts at a sun of its
    // own (its index modulo the group), so the suns' counters share the claims of the moment.
    const int32_t q0 = (int32_t)blockIdx.x % ng;
    for (int32_t qq = 0; qq < ng; qq++) {
        const int32_t q = (q0 + qq) % ng;
        const GroupSun& S = grp->sun[q];
        const int32_t n_items = S.bb.list_ctr[0];
        const int32_t n_large = ctr[S.s].n_large;
        const int32_t n_lc = min(n_large, kLargeCache);
        // light tiles (the list's tail) go one wave each when the sample fractions are in LDS and
        // the large list is short enough for a wave's slots
        const int32_t light = (TS == 64 && n_large <= kLargeCache && lds_tables) ? S.bb.list_ctr[2] : n_items;
        if (light == 0) continue;
        __syncthreads();                              // the previous sun's items are done with the cache
        static_assert(sizeof(TriRec) % 16 == 0, "records copy in 16-byte pieces");
        constexpr int kPieces = sizeof(TriRec) / 16;
        for (int32_t u = threadIdx.x; u < n_lc * kPieces; u += 256)
            reinterpret_cast<uint4*>(L.lcache)[u] =
                reinterpret_cast<const uint4*>(S.bb.rec + S.bb.large[u / kPieces])[u % kPieces];
        __syncthreads();
        for (;;) {
            if (threadIdx.x == 0) take = atomicAdd(&S.bb.list_ctr[1], 1);
            __syncthreads();
            const int32_t it = take;
            __syncthreads();
            if (it >= light) break;                   // the rest are the light pass's
            tile_body<TS, CAP>(L, S.bb.tile_list[it], n_lc, lds_tables, views[S.s], S.bb, n_large, n, S.g,
                               bias + S.s * S.g.n_mod, fu_tab, fv_tab, k, S.out, S.out.sparse, S.tmask);
            __syncthreads();
        }
    }
    if constexpr (TS == 64) {
        if (!lds_tables) return;
        __syncthreads();                              // the fraction tables are in place (no barrier above when no sun had heavy items)
        const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
        TriSlot* slots = reinterpret_cast<TriSlot*>(L.pool) + wv * kWaveSlots;
        const int32_t x0 = xcc_id();
        for (int32_t qq = 0; qq < ng; qq++) {
            const int32_t q = (q0 + qq) % ng;
            const GroupSun& S = grp->sun[q];
            const int32_t n_items = S.bb.list_ctr[0];
            if (ctr[S.s].n_large > kLargeCache) continue;   // every item was the workgroups'
            const int32_t light = S.bb.list_ctr[2];
            // the light items from their XCD sub-lists
            const int32_t n_light = n_items - light;
            const int32_t per_sub = (n_light + kXcds - 1) / kXcds;
            const int32_t claim = min(kLightClaimMax, max(kLightClaimMin, (per_sub + kLightPerClaim - 1) / kLightPerClaim));
            for (int32_t d = 0; d < kXcds; d++) {
                const int32_t j = (x0 + d) % kXcds;
                const int32_t n_j = n_light > j ? (n_light - j + kXcds - 1) / kXcds : 0;   // items light + j + kXcds i
                int32_t* const ctr_j = &S.bb.list_ctr[kXcdStride * (j + 1)];
                if (ld_dev(ctr_j) >= n_j) continue;           // taken already: no atomic
                int32_t got = 0;
                if (lane == 0) got = atomicAdd(ctr_j, claim);
                int32_t my0 = __builtin_amdgcn_readfirstlane(got);
                while (my0 < n_j) {
                    const int32_t my1 = min(my0 + claim, n_j);
                    // the next claim goes out with the claim's last tile, so that its round trip
                    // overlaps the tile's own reads (none when this claim reached the end)
                    for (int32_t i = my0; i < my1; i++) {
                        if (i == my1 - 1 && my1 < n_j && lane == 0) got = atomicAdd(ctr_j, claim);
                        wave_tile<TS>(slots, S.bb.tile_list[light + j + kXcds * i] >> 3, views[S.s], S.bb, ctr[S.s].n_large,
                                      n, S.g, bias + S.s * S.g.n_mod, L.ftab, L.ftab + knu, k, S.out, lane);
                    }
                    if (my1 == n_j) break;
                    my0 = __builtin_amdgcn_readfirstlane(got);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// depth check of the sub-cell samples (Fig. 4), one wave per cell
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sample_test(int64_t s, const View* views, GenDev g,
                                                     const double* beam, const int32_t* bias,
                                                     const double* fu_tab, const double* fv_tab, int32_t k,
                                                     const uint32_t* map, int32_t n, uint32_t* counts,
                                                     uint32_t* bits) {
    (void)beam;
    const int lane = threadIdx.x & 63;
    const int32_t cpm = g.n_cu * g.n_cv;
    const int64_t cell = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (cell >= (int64_t)g.n_mod * cpm) return;
    const int32_t m = (int32_t)(cell / cpm), c = (int32_t)(cell % cpm);
    const int32_t cu = c % g.n_cu, cv = c / g.n_cu;
    const int32_t kk = k * k, words = (kk + 31) / 32;
    uint32_t* cb = bits ? bits + cell * words : nullptr;
    const View& V = views[s];
    const int32_t bm = bias[s * g.n_mod + m];
    if (!V.valid || bm < 0) {
        if (lane == 0) counts[cell] = 0;
        if (cb)
            for (int w = lane; w < words; w += 64) cb[w] = 0;
        return;
    }
    const Module& M = g.mods[m];
    const d3 e1 = ld3(V.e1), e2 = ld3(V.e2), dd = ld3(V.d);
    const d3 p0 = to_light(V, ld3(M.o));
    const d3 U = ld3(M.u), W = ld3(M.v);
    const d3 du{dot(U, e1) * V.itx, dot(U, e2) * V.ity, dot(U, dd) * V.izd};
    const d3 dv{dot(W, e1) * V.itx, dot(W, e2) * V.ity, dot(W, dd) * V.izd};
    uint32_t cnt = 0;
    for (int32_t t0 = 0; t0 < kk; t0 += 64) {
        const int32_t t = t0 + lane;
        bool shaded = false;
        if (t < kk) {
            const int32_t a = t % k, b = t / k;
            const double fu = fu_tab[k * cu + a], fv = fv_tab[k * cv + b];
            const double x = (p0.x + fu * du.x) + fv * dv.x;
            const double y = (p0.y + fu * du.y) + fv * dv.y;
            const double z = (p0.z + fu * du.z) + fv * dv.z;
            int64_t i = (int64_t)floor(x), j = (int64_t)floor(y);
            const int64_t zs = (int64_t)floor(z);
            i = min(max(i, (int64_t)0), (int64_t)n - 1);
            j = min(max(j, (int64_t)0), (int64_t)n - 1);
            shaded = zs > (int64_t)map[j * n + i] + (int64_t)bm;
        }
        const uint64_t bal = __ballot(shaded);
        cnt += (uint32_t)__popcll(bal);
        if (cb && lane == 0) {
            const int32_t w = t0 / 32;
            cb[w] = (uint32_t)bal;
            if (w + 1 < words) cb[w + 1] = (uint32_t)(bal >> 32);
        }
    }
    if (lane == 0) counts[cell] = cnt;
}

// ---------------------------------------------------------------------------
// Step 4: ideal bypass-diode strings, one workgroup per sun
// ---------------------------------------------------------------------------
constexpr int kMaxSubPerString = 4096;

constexpr int kLossStrings = 1024;   // strings per chunk of the loss

struct LossLds {
    double cap[kMaxSubPerString];        // substring capacities of a chunk of whole strings
    double best[kLossStrings];           // best operating point of each string of the chunk
    int32_t chunk[2];                    // [first string, end string) of the chunk
};

// ---------------------------------------------------------------------------
// Step 4 with the single-diode cell model: every cell follows
//   I = Iph - I0 (exp((V + I Rs) / a) - 1) - (V + I Rs) / Rsh,  Iph = isc G / gref,
// a substring's bypass diode keeps its voltage at -vb or above, substrings are
// in series, and each string works at its maximum power point. One wave per
// string; lanes take the string's substrings.
// ---------------------------------------------------------------------------
constexpr int kDiodeCells = 2048;     // shaded counts of one string staged per wave
constexpr int kDiodeLevels = 128;     // slots of the level route's voltage table: two per lane
constexpr int kDiodeStrings = 512;    // strings per chunk of the single-diode loss
constexpr int kMppGrid = 64;          // current grid of the maximum power search
constexpr int kMppRefine = 40;        // golden-section steps around each grid maximum

struct DiodeLds {
    uint16_t cnt[4][kDiodeCells];     // per wave: its string's counts (level ranks on the level route),
                                      // module by module, substring-major
    unsigned long long rk[4][4][64];  // per wave: each lane's cells' level ranks, eight to a word, word-major
    double vt[4][kDiodeLevels];       // per wave: the level route's voltage table
    double spow[2][kDiodeStrings];    // shaded and unshaded powers of a chunk of strings
};

// Orders a wave's LDS stores before its own later loads from other lanes (one
// wave: no workgroup barrier).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Cell voltage at current I and irradiance G. In the diode voltage x = V + I Rs
// the equation is f(x) = c - I0 exp(x / a) - x / Rsh = 0 with c = Iph + I0 - I;
// f falls and is concave, so Newton's method from a point where f <= 0 moves
// down to the root without passing it. Start: the smaller of Rsh c (where
// f = -I0 exp(x / a)) and, when c >= I0, a ln(c / I0) (where f = -x / Rsh). The
// iteration ends when a step no longer lowers x.
__device__ double cell_voltage(const DiodeDev& d, double G, double I) {
    const double iph = d.isc * G / d.gref;
    const double c = iph + d.i0 - I;
    double x = d.rsh * c;
    if (c >= d.i0) {
        const double xl = d.a * log(c / d.i0);
        if (xl < x) x = xl;
    }
    for (int it = 0; it < 64; it++) {
        const double e = exp(x / d.a);
        const double f = (c - d.i0 * e) - x / d.rsh;
        const double fp = -(d.i0 / d.a) * e - 1.0 / d.rsh;
        const double xn = x - f / fp;
        if (!(xn < x)) break;
        x = xn;
    }
    return x - I * d.rs;
}

// Sum over the wave, the same value in every lane (pairs add commutatively).
__device__ __forceinline__ double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One string of one sun, as one wave sees it.
struct DiodeString {
    const GenDev* g;
    const double* beam_s;         // per-module beam of the sun
    const uint32_t* counts_s;     // per-cell shaded counts (nullptr: none shaded)
    uint16_t* staged;             // the string's counts staged in LDS, or nullptr
    unsigned long long* rk;       // the wave's rank words in LDS ([4][64])
    double* vt;                   // the wave's table of level voltages in LDS
    const double* svf;            // per-cell sky view factors, or nullptr (whole sky)
    double dp, kk;                // diffuse irradiance, samples per cell
    int32_t p0, nq, cpm;          // first module of the string in str_mods, substrings, cells per module
};

// Shaded count of the i-th cell (in substring order) of the string's mi-th module.
template <bool COHERENT>
__device__ __forceinline__ int32_t diode_count(const DiodeString& S, int32_t mi, int32_t m, int32_t i) {
    if (S.staged) return S.staged[mi * S.cpm + i];
    if (!S.counts_s) return 0;
    const uint32_t* p = S.counts_s + (int64_t)m * S.cpm + S.g->sub_cell[i];
    return (int32_t)(COHERENT ? ld_dev(p) : *p);
}

// Irradiance of that cell: the beam on its module minus the shaded share, plus
// the diffuse times the share of the sky the cell sees (whole sky: reference).
template <bool COHERENT>
__device__ __forceinline__ double diode_irradiance(const DiodeString& S, int32_t mi, int32_t m, int32_t i, double bm) {
    const int32_t cn = diode_count<COHERENT>(S, mi, m, i);
    const double sky = S.svf ? S.svf[(int64_t)m * S.cpm + S.g->sub_cell[i]] : 1.0;
    return bm * (1.0 - (double)cn / S.kk) + S.dp * sky;
}

// Voltage of substring q of the string at current I: its cells in order, one
// solve per run of equal irradiances, clamped by the bypass diode.
template <bool COHERENT>
__device__ double sub_voltage(const DiodeString& S, int32_t q, double I) {
    const GenDev& g = *S.g;
    const int32_t mi = q / g.n_sub, sq = q % g.n_sub;
    const int32_t m = g.str_mods[S.p0 + mi];
    const double bm = S.beam_s[m];
    double vs = 0.0, vc = 0.0, prev = -1.0;
    for (int32_t i = g.sub_start[sq]; i < g.sub_start[sq + 1]; i++) {
        const double G = diode_irradiance<COHERENT>(S, mi, m, i, bm);
        if (G != prev) {
            vc = cell_voltage(g.diode, G, I);
            prev = G;
        }
        vs += vc;
    }
    return vs < -g.diode.vb ? -g.diode.vb : vs;
}

// Levels of a string whose cells differ only by their shaded count (one beam
// for all its modules, no sky view factors, at most 128 counts): the counts
// present, as a 128-bit mask the whole wave holds. The wave's table has 128
// slots, two per lane (lane and lane + 64); slot s holds the cell voltage of
// level s % n at the (s / n)-th current of a batch, so that one round of
// solves serves 128 / n currents, and every level is solved once per current
// instead of wherever some lane's irradiance changes. Each cell then reads its
// level's value from the table. The values, and the order in which cells add
// up, are those of sub_voltage.
struct Levels {
    unsigned long long m0, m1;    // counts 0..63 and 64..127 present in the string
    double g0, g1;                // irradiances of the lane's two slots' levels
    int32_t n;                    // levels
    int32_t c0, c1;               // the lane's two slots' currents within a batch
    int32_t maxc;                 // most cells of a substring
    int32_t nc;                   // cells of the lane's substring when ranks are in words (0: none)
    bool on, words;               // level route; ranks in words (at most 64 substrings of at most 32 cells)
};

__device__ __forceinline__ int32_t level_rank(const Levels& L, int32_t cn) {
    return cn < 64 ? __popcll(L.m0 & ((1ull << cn) - 1ull))
                   : __popcll(L.m0) + __popcll(L.m1 & ((1ull << (cn - 64)) - 1ull));
}

// The count of level r (r < n): the r-th set bit of the mask.
__device__ int32_t level_count(const Levels& L, int32_t r) {
    const int32_t n0 = __popcll(L.m0);
    unsigned long long m = r < n0 ? L.m0 : L.m1;
    for (int32_t t = r < n0 ? r : r - n0; t > 0; t--) m &= m - 1ull;
    return (r < n0 ? 0 : 64) + __builtin_ctzll(m);
}

// The string's levels. On the level route, staged counts become level ranks
// (each lane converts the cells of its own substrings, the only ones it reads),
// and a string of at most 64 substrings of at most 32 cells also packs each
// lane's ranks into words, so that a lane reads eight cells' ranks at once.
template <bool COHERENT>
__device__ void string_levels(const DiodeString& S, int lane, Levels& L) {
    const GenDev& g = *S.g;
    L.on = L.words = false;
    L.n = L.c0 = L.c1 = L.maxc = L.nc = 0;
    L.g0 = L.g1 = 0.0;
    L.m0 = L.m1 = 0ull;
    if (S.svf || S.kk > 127.5) return;                                  // uniform over the wave
    double bmin = INFINITY, bmax = -INFINITY;
    int32_t maxc = 0;
    for (int32_t q = lane; q < S.nq; q += 64) {
        const int32_t mi = q / g.n_sub, sq = q % g.n_sub;
        const int32_t m = g.str_mods[S.p0 + mi];
        const double bm = S.beam_s[m];
        bmin = fmin(bmin, bm);
        bmax = fmax(bmax, bm);
        maxc = max(maxc, g.sub_start[sq + 1] - g.sub_start[sq]);
        for (int32_t i = g.sub_start[sq]; i < g.sub_start[sq + 1]; i++) {
            const int32_t cn = diode_count<COHERENT>(S, mi, m, i);
            if (cn < 64) L.m0 |= 1ull << cn;
            else L.m1 |= 1ull << (cn - 64);
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        bmin = fmin(bmin, __shfl_xor(bmin, off, 64));
        bmax = fmax(bmax, __shfl_xor(bmax, off, 64));
        maxc = max(maxc, __shfl_xor(maxc, off, 64));
        L.m0 |= __shfl_xor(L.m0, off, 64);
        L.m1 |= __shfl_xor(L.m1, off, 64);
    }
    L.n = __popcll(L.m0) + __popcll(L.m1);
    if (!(bmin == bmax)) return;
    L.on = true;
    L.maxc = maxc;
    L.c0 = lane / L.n;
    L.c1 = (lane + 64) / L.n;
    // as diode_irradiance forms them
    L.g0 = bmin * (1.0 - (double)level_count(L, lane % L.n) / S.kk) + S.dp * 1.0;
    L.g1 = bmin * (1.0 - (double)level_count(L, (lane + 64) % L.n) / S.kk) + S.dp * 1.0;
    if (S.staged)
        for (int32_t q = lane; q < S.nq; q += 64) {
            const int32_t mi = q / g.n_sub, sq = q % g.n_sub;
            for (int32_t i = g.sub_start[sq]; i < g.sub_start[sq + 1]; i++) {
                uint16_t& c = S.staged[mi * S.cpm + i];
                c = (uint16_t)level_rank(L, c);
            }
        }
    L.words = S.nq <= 64 && maxc <= 32;
    if (!L.words || lane >= S.nq) return;
    const int32_t mi = lane / g.n_sub, sq = lane % g.n_sub;
    const int32_t m = g.str_mods[S.p0 + mi];
    const int32_t c0 = g.sub_start[sq];
    L.nc = g.sub_start[sq + 1] - c0;
    for (int32_t w = 0; 8 * w < L.nc; w++) {
        unsigned long long word = 0ull;
        for (int32_t t = 0; t < 8 && 8 * w + t < L.nc; t++) {
            const int32_t i = c0 + 8 * w + t;
            const unsigned long long r = S.staged ? (unsigned long long)S.staged[mi * S.cpm + i]
                                                  : (unsigned long long)level_rank(L, diode_count<COHERENT>(S, mi, m, i));
            word |= r << (8 * t);
        }
        S.rk[w * 64 + lane] = word;
    }
}

// The lane's share of the string voltage on the level route, its cells reading
// the table from slot o on: the sum of its substrings' clamped voltages.
template <bool COHERENT>
__device__ __forceinline__ double level_volts(const DiodeString& S, const Levels& L, int32_t lane, int32_t o) {
    const GenDev& g = *S.g;
    const double* vt = S.vt + o;
    if (L.words) {
        if (L.nc == 0) return 0.0;
        double vs = 0.0;
        for (int32_t w = 0; 8 * w < L.nc; w++) {
            const unsigned long long word = S.rk[w * 64 + lane];
            double x[8];
#pragma unroll
            for (int t = 0; t < 8; t++) x[t] = vt[(word >> (8 * t)) & 0xffull];    // past the end: rank 0
#pragma unroll
            for (int t = 0; t < 8; t++) vs = 8 * w + t < L.nc ? vs + x[t] : vs;
        }
        return vs < -g.diode.vb ? -g.diode.vb : vs;
    }
    double v = 0.0;
    for (int32_t q = lane; q < S.nq; q += 64) {
        const int32_t mi = q / g.n_sub, sq = q % g.n_sub;
        const int32_t m = g.str_mods[S.p0 + mi];
        double vs = 0.0;
        for (int32_t i = g.sub_start[sq]; i < g.sub_start[sq + 1]; i++)
            vs += vt[S.staged ? (int32_t)S.staged[mi * S.cpm + i] : level_rank(L, diode_count<COHERENT>(S, mi, m, i))];
        vs = vs < -g.diode.vb ? -g.diode.vb : vs;
        v += vs;
    }
    return v;
}

// String power at current I.
template <bool COHERENT>
__device__ double string_power_at(const DiodeString& S, const Levels& L, int lane, double I) {
    if (!L.on) {
        double v = 0.0;
        for (int32_t q = lane; q < S.nq; q += 64) v += sub_voltage<COHERENT>(S, q, I);
        return I * wave_sum(v);
    }
    const GenDev& g = *S.g;
    if (lane < L.n) S.vt[lane] = cell_voltage(g.diode, L.g0, I);
    if (lane + 64 < L.n) S.vt[lane + 64] = cell_voltage(g.diode, L.g1, I);
    wave_lds_sync();
    const double v = level_volts<COHERENT>(S, L, lane, 0);
    wave_lds_sync();                                  // the table is rewritten at the next current
    return I * wave_sum(v);
}

// Maximum power of the string over currents [0, Imax], Imax its largest cell
// photocurrent: the power at kMppGrid + 1 evenly spaced currents, then a
// golden-section search over the two grid steps around every sample that is
// not below its neighbours; the largest value seen, at least 0. Every lane
// holds the same powers, so the search's branches are uniform. The grid powers
// come first (in batches on the level route), lane j keeping the j-th; the
// largest value seen does not depend on the order in which values are seen. A
// string on the level route whose only count is 0 has the inputs of its
// unshaded self: with that power known (has_clear), the search returns it.
template <bool COHERENT>
__device__ double string_mpp_wave(const DiodeString& S, int lane, bool has_clear, double clear) {
    const GenDev& g = *S.g;
    const DiodeDev& d = g.diode;
    double imax = 0.0;
    for (int32_t q = lane; q < S.nq; q += 64) {
        const int32_t mi = q / g.n_sub, sq = q % g.n_sub;
        const int32_t m = g.str_mods[S.p0 + mi];
        const double bm = S.beam_s[m];
        for (int32_t i = g.sub_start[sq]; i < g.sub_start[sq + 1]; i++) {
            const double iph = d.isc * diode_irradiance<COHERENT>(S, mi, m, i, bm) / d.gref;
            imax = fmax(imax, iph);
        }
    }
    for (int off = 32; off > 0; off >>= 1) imax = fmax(imax, __shfl_xor(imax, off, 64));
    if (!(imax > 0.0)) return 0.0;
    Levels L;
    string_levels<COHERENT>(S, lane, L);
    if (has_clear && L.on && L.n == 1 && L.m0 == 1ull) return clear;
    // grid powers: lane j holds the power at current j Imax / kMppGrid (j < kMppGrid), gtop at Imax
    double gp = 0.0, gtop = 0.0;
    if (L.on) {
        const int32_t per = min(kMppGrid + 1, kDiodeLevels / L.n);     // currents per round of solves
        for (int32_t base = 0; base <= kMppGrid; base += per) {
            const int32_t nb = min(per, kMppGrid + 1 - base);
            if (L.c0 < nb) S.vt[lane] = cell_voltage(d, L.g0, imax * (double)(base + L.c0) / (double)kMppGrid);
            if (L.c1 < nb) S.vt[lane + 64] = cell_voltage(d, L.g1, imax * (double)(base + L.c1) / (double)kMppGrid);
            wave_lds_sync();
            for (int32_t c = 0; c < nb; c++) {
                const int32_t q = base + c;
                const double p = imax * (double)q / (double)kMppGrid * wave_sum(level_volts<COHERENT>(S, L, lane, c * L.n));
                if (q == lane) gp = p;
                if (q == kMppGrid) gtop = p;
            }
            wave_lds_sync();
        }
    } else {
        for (int32_t q = 0; q <= kMppGrid; q++) {
            const double p = string_power_at<COHERENT>(S, L, lane, imax * (double)q / (double)kMppGrid);
            if (q == lane) gp = p;
            if (q == kMppGrid) gtop = p;
        }
    }
    const double r = 0.6180339887498949;       // (sqrt(5) - 1) / 2
    double best = 0.0;
    for (int q = 1; q <= kMppGrid; q++) {
        const double pm = __shfl(gp, q - 1, 64);
        const double pc = q < kMppGrid ? __shfl(gp, q, 64) : gtop;
        const double pn = q < kMppGrid - 1 ? __shfl(gp, q + 1, 64) : gtop;
        if (pc >= pm && (q == kMppGrid || pc >= pn)) {
            if (pc > best) best = pc;
            double lo = imax * (double)(q - 1) / (double)kMppGrid;
            double hi = imax * (double)(q < kMppGrid ? q + 1 : q) / (double)kMppGrid;
            double xc = hi - r * (hi - lo), xd = lo + r * (hi - lo);
            double fc = 0.0, fd = 0.0;
            // the two inner points, then kMppRefine steps, each evaluating the point it moves
            for (int it = -2; it < kMppRefine; it++) {
                bool left;
                double x;
                if (it == -2) {
                    x = xc; left = true;
                } else if (it == -1) {
                    x = xd; left = false;
                } else if (fc >= fd) {
                    hi = xd; xd = xc; fd = fc;
                    xc = hi - r * (hi - lo);
                    x = xc; left = true;
                } else {
                    lo = xc; xc = xd; fc = fd;
                    xd = lo + r * (hi - lo);
                    x = xd; left = false;
                }
                const double f = string_power_at<COHERENT>(S, L, lane, x);
                if (left) fc = f;
                else fd = f;
                if (f > best) best = f;
            }
        }
    }
    return best;
}

// One sun with the single-diode model: strings in chunks of kDiodeStrings, a
// wave per string for its unshaded power (the reference) and then its shaded
// power, the powers of each kind added in string order. The unshaded power of
// a string whose modules share one beam depends only on its module count and
// that beam: the wave reuses its previous such string's power when both match
// (the same inputs to the same computation, so the same value).
template <bool COHERENT>
__device__ void diode_loss_body(DiodeLds& L, const double* beam_s, const uint32_t* counts_s, double dp,
                                const GenDev& g, int32_t k, double* power_s, double* power_ref_s) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int32_t cpm = g.n_cu * g.n_cv;
    double tot[2] = {0.0, 0.0};
    int32_t ref_nm = -1;                      // the wave's last uniform-beam string: modules, beam, power
    double ref_bm = 0.0, ref_p = 0.0;
    for (int32_t st0 = 0; st0 < g.n_str; st0 += kDiodeStrings) {
        const int32_t st1 = min(g.n_str, st0 + kDiodeStrings);
        for (int32_t st = st0 + wv; st < st1; st += 4) {
            DiodeString S;
            S.g = &g;
            S.beam_s = beam_s;
            S.counts_s = nullptr;
            S.staged = nullptr;
            S.rk = &L.rk[wv][0][0];
            S.vt = L.vt[wv];
            S.svf = nullptr;
            S.dp = dp;
            S.kk = (double)(k * k);
            S.p0 = g.str_start[st];
            S.cpm = cpm;
            const int32_t nm = g.str_start[st + 1] - S.p0;
            S.nq = nm * g.n_sub;
            double bmin = INFINITY, bmax = -INFINITY;
            for (int32_t mi = lane; mi < nm; mi += 64) {
                const double bm = beam_s[g.str_mods[S.p0 + mi]];
                bmin = fmin(bmin, bm);
                bmax = fmax(bmax, bm);
            }
            for (int off = 32; off > 0; off >>= 1) {
                bmin = fmin(bmin, __shfl_xor(bmin, off, 64));
                bmax = fmax(bmax, __shfl_xor(bmax, off, 64));
            }
            const bool uni = bmin == bmax;
            double pu;
            if (uni && nm == ref_nm && bmin == ref_bm) {
                pu = ref_p;
            } else {
                pu = string_mpp_wave<COHERENT>(S, lane, false, 0.0);
                ref_nm = uni ? nm : -1;
                ref_bm = bmin;
                ref_p = pu;
            }
            S.counts_s = counts_s;
            S.svf = g.svf;
            if (nm * cpm <= kDiodeCells) {
                // each lane stages the cells of its own substrings, and reads only those
                uint16_t* dst = L.cnt[wv];
                for (int32_t q = lane; q < S.nq; q += 64) {
                    const int32_t mi = q / g.n_sub, sq = q % g.n_sub;
                    const int32_t m = g.str_mods[S.p0 + mi];
                    for (int32_t i = g.sub_start[sq]; i < g.sub_start[sq + 1]; i++)
                        dst[mi * cpm + i] = (uint16_t)diode_count<COHERENT>(S, mi, m, i);
                }
                S.staged = dst;
            }
            const double ps = string_mpp_wave<COHERENT>(S, lane, true, pu);
            if (lane == 0) {
                L.spow[0][st - st0] = ps;
                L.spow[1][st - st0] = pu;
            }
        }
        __syncthreads();
        if (tid == 0)
            for (int32_t st = st0; st < st1; st++) {
                tot[0] += L.spow[0][st - st0];
                tot[1] += L.spow[1][st - st0];
            }
        __syncthreads();
    }
    if (tid == 0) {
        *power_s = tot[0];
        *power_ref_s = tot[1];
    }
}

// One sun: sun3 its unit vector, beam_s its per-module beam, counts_s its
// per-cell shaded counts, dp its diffuse irradiance. Strings go in chunks
// (consecutive whole strings, at most kMaxSubPerString substrings): every
// substring capacity of the chunk at once, then one wave per string for its
// best current, then the string powers added in string order.
template <bool COHERENT>
__device__ void loss_body(LossLds& L, const double* sun3, const double* beam_s, const uint32_t* counts_s, double dp,
                          const GenDev& g, int32_t k, double* power_s, double* power_ref_s) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    if (!(sun3[2] > 0.0)) {
        if (tid == 0) { *power_s = 0.0; *power_ref_s = 0.0; }
        return;
    }
    if (g.diode.on) {
        static_assert(sizeof(DiodeLds) <= sizeof(LossLds), "the diode model works in the loss stage's LDS");
        diode_loss_body<COHERENT>(*reinterpret_cast<DiodeLds*>(&L), beam_s, counts_s, dp, g, k, power_s, power_ref_s);
        return;
    }
    const int32_t cpm = g.n_cu * g.n_cv;
    const double kk = (double)(k * k);
    double tot[2] = {0.0, 0.0};
    for (int32_t st0 = 0; st0 < g.n_str;) {
        if (tid == 0) {
            int32_t st1 = st0;
            while (st1 < g.n_str && st1 - st0 < kLossStrings &&
                   (g.str_start[st1 + 1] - g.str_start[st0]) * g.n_sub <= kMaxSubPerString)
                st1++;
            L.chunk[0] = st0;
            L.chunk[1] = st1;
        }
        __syncthreads();
        const int32_t st1 = L.chunk[1];
        const int32_t p0 = g.str_start[st0];
        const int32_t nq = (g.str_start[st1] - p0) * g.n_sub;
        for (int pass = 0; pass < 2; pass++) {
            for (int32_t q = tid; q < nq; q += 256) {
                const int32_t m = g.str_mods[p0 + q / g.n_sub], sq = q % g.n_sub;
                const double bm = beam_s[m];
                double cmin = INFINITY;
                for (int32_t i = g.sub_start[sq]; i < g.sub_start[sq + 1]; i++) {   // the substring's cells
                    const int32_t c = g.sub_cell[i];
                    const uint32_t sh = pass == 0 ? (COHERENT ? ld_dev(counts_s + (int64_t)m * cpm + c)
                                                              : counts_s[(int64_t)m * cpm + c])
                                                  : 0u;
                    const double f = (double)sh / kk;
                    const double sky = pass == 0 && g.svf ? g.svf[(int64_t)m * cpm + c] : 1.0;
                    cmin = fmin(cmin, bm * (1.0 - f) + dp * sky);
                }
                L.cap[q] = cmin;
            }
            __syncthreads();
            for (int32_t st = st0 + wv; st < st1; st += 4) {
                const int32_t a = (g.str_start[st] - p0) * g.n_sub, b = (g.str_start[st + 1] - p0) * g.n_sub;
                double best = 0.0;
                for (int32_t q = a + lane; q < b; q += 64) {
                    const double v = L.cap[q];
                    int32_t cnt = 0;
                    for (int32_t r = a; r < b; r++) cnt += L.cap[r] >= v ? 1 : 0;
                    best = fmax(best, (double)cnt * v);
                }
                for (int off = 32; off > 0; off >>= 1) best = fmax(best, __shfl_xor(best, off, 64));
                if (lane == 0) L.best[st - st0] = best;
            }
            __syncthreads();
            if (tid == 0)
                for (int32_t st = st0; st < st1; st++) tot[pass] += L.best[st - st0];
            __syncthreads();
        }
        st0 = st1;
    }
    if (tid == 0) {
        *power_s = tot[0];
        *power_ref_s = tot[1];
    }
}

// A sun whose set-up records or bin entries overflowed their buffers (never
// with the per-sun path's capacities; a guard all the same) reads NaN powers,
// so a caller of the asynchronous form sees it without a host round trip.
__global__ __launch_bounds__(256, 3) void k_loss(int64_t s0, const double* sun, const double* beam,
                                              const uint32_t* counts, const double* d_poa, GenDev g, int32_t k,
                                              double* power, double* power_ref, const SunCounters* ctr) {
    __shared__ LossLds L;
    const int64_t s = s0 + blockIdx.x;
    const int64_t n_cells = (int64_t)g.n_mod * g.n_cu * g.n_cv;
    loss_body<false>(L, sun + 3 * s, beam + s * g.n_mod, counts + s * n_cells, d_poa[s], g, k, power + s, power_ref + s);
    if (ctr && threadIdx.x == 0 && ctr[s].overflow) {
        power[s] = __builtin_nan("");
        power_ref[s] = __builtin_nan("");
    }
}

// The sums over suns, in sun order by one thread; the workgroup stages the
// arrays in LDS a chunk at a time, so that the sequential sum reads LDS
// instead of waiting on a global load per sun.
constexpr int kEnergyChunk = 1024;
__global__ __launch_bounds__(256) void k_energy(int64_t n_sun, const double* power, const double* power_ref,
                                                const double* dt, double* energy) {
    __shared__ double pw[kEnergyChunk], pr[kEnergyChunk], dl[kEnergyChunk];
    double e = 0.0, er = 0.0;
    for (int64_t t0 = 0; t0 < n_sun; t0 += kEnergyChunk) {
        const int32_t m = (int32_t)min<int64_t>(kEnergyChunk, n_sun - t0);
        for (int32_t i = threadIdx.x; i < m; i += blockDim.x) {
            pw[i] = power[t0 + i];
            pr[i] = power_ref[t0 + i];
            dl[i] = dt[t0 + i];
        }
        __syncthreads();
        if (threadIdx.x == 0)
            for (int32_t i = 0; i < m; i++) {
                e += pw[i] * dl[i];
                er += pr[i] * dl[i];
            }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        energy[0] = e;
        energy[1] = er;
    }
}

// Diffuse shading: sky view factor of every cell from the shaded counts of
// n_dir sky directions (each evaluated as a sun): the front-facing directions'
// weights w = n . s, in direction order, times the cell's lit share, over the
// sum of the weights; 1 when no direction faces the module.
__global__ __launch_bounds__(256) void k_svf(const Module* mods, int32_t cpm, int64_t n_cells, const double* dirs,
                                             int64_t n_dir, const uint32_t* counts, int32_t k, double* svf) {
    const int64_t c = blockIdx.x * 256ll + threadIdx.x;
    if (c >= n_cells) return;
    const Module& M = mods[c / cpm];
    const double kk = (double)(k * k);
    double num = 0.0, den = 0.0;
    for (int64_t j = 0; j < n_dir; j++) {
        const double w = (M.n[0] * dirs[3 * j] + M.n[1] * dirs[3 * j + 1]) + M.n[2] * dirs[3 * j + 2];
        if (!(w > 0.0)) continue;
        const double f = (double)counts[j * n_cells + c] / kk;
        num += w * (1.0 - f);
        den += w;
    }
    svf[c] = den > 0.0 ? num / den : 1.0;
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = v;
}

// ---------------------------------------------------------------------------
// persistent launch: workgroups take units of (job, sun) items from per-slot
// queues until every item is done. The units run the same bodies as the
// per-sun kernels above, so results are the same.
// ---------------------------------------------------------------------------
constexpr size_t cmax(size_t a, size_t b) { return a > b ? a : b; }
constexpr size_t kPLdsBytes = cmax(cmax(sizeof(TileLds<64, kCap64>), sizeof(TileLds<32, kCap32>)),
                                   cmax(cmax(sizeof(SetupLds), sizeof(LossLds)), (2 * 256 + 2 * kScanBuckets) * 4 + 1024 * 8));

__device__ __forceinline__ unsigned long long pword(int32_t phase, int32_t n_units) {
    return ((unsigned long long)(uint32_t)phase << 56) | ((unsigned long long)(uint32_t)n_units << 32);
}
__device__ __forceinline__ int32_t w_phase(unsigned long long w) { return (int32_t)(w >> 56); }
__device__ __forceinline__ uint32_t w_units(unsigned long long w) { return (uint32_t)(w >> 32) & 0xFFFFFFu; }
__device__ __forceinline__ uint32_t w_next(unsigned long long w) { return (uint32_t)w; }
__device__ __forceinline__ bool w_open(unsigned long long w) { return w_phase(w) != kPhIdle && w_next(w) < w_units(w); }

__device__ __forceinline__ BinBuffers slot_bins(const PLaunch& P, const PJob& J, const PSlotBufs& B) {
    BinBuffers bb;
    bb.rec = B.rec;
    bb.rec_cap = P.rec_cap;
    bb.large = B.large;
    bb.tile_count = B.tile_count;
    bb.tile_start = B.tile_start;
    bb.tile_cursor = B.tile_cursor;
    bb.bins = B.bins;
    bb.modbox = B.modbox;
    bb.tile_list = nullptr;           // the scan and tile units use the slot's list directly
    bb.list_ctr = nullptr;
    bb.split_at = 0;
    bb.pitems = nullptr;              // units count their pairs as they set up
    bb.pchunk = nullptr;
    bb.pctr = nullptr;
    bb.item_cap = 0;
    bb.bin_cap = P.bin_cap;
    bb.tile = J.tile;
    bb.ntx = J.ntx;
    bb.n_tiles = J.n_tiles;
    bb.large_tiles = J.large_tiles;
    return bb;
}

// The job's generator as one sun sees it: trackers' modules posed for that sun.
__device__ __forceinline__ GenDev sun_gen(const PJob& J, const PItem it) {
    GenDev g = J.g;
    if (g.mods_sun) g.mods = g.mods_sun + (int64_t)it.sun * g.n_mod;
    return g;
}

// Each phase as a function of its own, so the persistent kernel needs the
// registers of its largest phase, not of all phases inlined together.
__device__ __noinline__ void unit_setup(unsigned char* raw, const PJob& J, const PItem it, const PSlotBufs& B) {
    if (threadIdx.x == 0) {                // counters other units update with atomics
        __hip_atomic_store(&B.ctr->n_rec, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&B.ctr->n_large, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&B.ctr->overflow, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    uint32_t* row = J.counts + (int64_t)it.sun * J.cells;     // tile units add to it with atomics
    for (int64_t c = threadIdx.x; c < J.cells; c += 256)
        __hip_atomic_store(row + c, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const TileGrid tg{J.tile, J.ntx, J.n_tiles, J.words};
    setup_body(*reinterpret_cast<SetupLds*>(raw), J.sun + 3 * it.sun, J.dni[it.sun], sun_gen(J, it), J.sphere, J.n,
               B.view, B.beam, B.bias, tg, J.use_mask ? B.tmask : nullptr);
}

__device__ __noinline__ void unit_tri(unsigned char* raw, const PJob& J, const PItem it, const PSlotBufs& B,
                                      const BinBuffers& bb, int32_t unit) {
    const int64_t total = J.sc.n_tri + (J.g.occluders ? 2 * (int64_t)J.g.n_mod : 0) + J.g.n_mod;
    const int64_t t0 = (int64_t)unit * kTriPerUnit;
    uint32_t* cnt = 4 * (size_t)J.n_tiles <= kPLdsBytes ? reinterpret_cast<uint32_t*>(raw) : nullptr;
    tri_setup_body(cnt, t0, min(t0 + kTriPerUnit, total), *B.view, J.sc, sun_gen(J, it), B.bias, J.n, bb, B.ctr,
                   J.use_mask ? B.tmask : nullptr);
}

__device__ __noinline__ void unit_scan(unsigned char* raw, const PLaunch& P, const PJob& J, const PSlotBufs& B,
                                       const BinBuffers& bb, PSlotState& st) {
    int32_t* part = reinterpret_cast<int32_t*>(raw);
    // tile order: a slot's workgroups sit on one XCD, and neighbouring tiles
    // share triangle records in its L2; the slots balance the load
    const int32_t n_list = scan_body<256, true>(part, J.n_tiles, bb, B.tile_list, -1);
    if (threadIdx.x == 0) {
        const int32_t total = part[0];
        const int32_t ovf = (ld_dev(&B.ctr->overflow) || ld_dev(&B.ctr->n_rec) > P.rec_cap || total > P.bin_cap) ? 1 : 0;
        __hip_atomic_store(&st.n_list, n_list, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&st.overflow, ovf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__device__ __noinline__ void unit_scatter(unsigned char* raw, const PJob& J, const PSlotBufs& B, const BinBuffers& bb,
                                          int32_t unit, int32_t units) {
    uint32_t* lds = 8 * (size_t)J.n_tiles <= kPLdsBytes ? reinterpret_cast<uint32_t*>(raw) : nullptr;
    scatter_body(lds, unit, units, bb, J.g.n_mod, ld_dev(&B.ctr->n_rec), B.ctr, J.use_mask ? B.tmask : nullptr);
}

__device__ __noinline__ void unit_tile(unsigned char* raw, const PJob& J, const PItem it, const PSlotBufs& B,
                                       const BinBuffers& bb, int32_t unit) {
    const int32_t item = B.tile_list[unit];
    const GenDev gs = sun_gen(J, it);
    TileOut out;
    out.map = nullptr;
    out.counts = J.counts + (int64_t)it.sun * J.cells;
    out.bits = nullptr;
    out.test = 1;
    out.sparse = J.sparse;
    const uint32_t* tmask = J.use_mask ? B.tmask : nullptr;
    if (J.tile == 64)
        tile_body<64, kCap64>(*reinterpret_cast<TileLds<64, kCap64>*>(raw), item, 0, false, *B.view, bb, ld_dev(&B.ctr->n_large), J.n, gs,
                            B.bias, J.fu, J.fv, J.k, out, J.sparse, tmask);
    else
        tile_body<32, kCap32>(*reinterpret_cast<TileLds<32, kCap32>*>(raw), item, 0, false, *B.view, bb, ld_dev(&B.ctr->n_large), J.n, gs,
                            B.bias, J.fu, J.fv, J.k, out, J.sparse, tmask);
}

__device__ __noinline__ void unit_loss(unsigned char* raw, const PJob& J, const PItem it, const PSlotBufs& B) {
    loss_body<true>(*reinterpret_cast<LossLds*>(raw), J.sun + 3 * it.sun, B.beam, J.counts + (int64_t)it.sun * J.cells,
              J.dpoa[it.sun], J.g, J.k, J.power + it.sun, J.power_ref + it.sun);
}

// Coherence of the persistent launch. Taking a unit is a device-scope
// acquire (this CU's L1 and the L2's non-coherent lines dropped, dirty lines
// kept), so a unit never reads a line cached before its inputs were written,
// even when a slot's buffers held another item a moment ago. With XCD
// groups, the units of a slot run on one XCD, whose L2 every producer and
// consumer of the slot's buffers share, so a unit's release only has to wait
// for its own stores; without groups it writes the L2 back to memory. Words
// that other units update with atomics are read with ld_dev.
__device__ __forceinline__ void acquire_unit(int32_t) { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

// s_waitcnt vmcnt(0) expcnt(7) lgkmcnt(15): every vector memory access of the wave done
constexpr int kWaitVmem = 0x0F70;
// Serving: workgroups that read the host's words, and how often (wall-clock ticks, 100 MHz).
constexpr int32_t kPollers = 8;
constexpr long long kPollTicks = 200;


struct PCtl {
    int32_t slot, unit, phase, units;
    int32_t stop, finish, job_last, job;
    int32_t count;          // units claimed at once: unit, unit + 1, ...
};

// Units of the many-unit phases (triangles, scatter, tiles) are claimed a
// quarter of the remaining ones at a time, at most kMaxClaim, and run one
// after the other: every claim is an atomic on the slot word that all of
// the XCD's workgroups contend for. One unit per claim spent about a third
// of the launch in claiming; the guided claim also keeps the last units of
// a phase small, so the item's next phase is not held up.
constexpr int32_t kMaxClaim = 32;
constexpr int32_t kClaimDiv = 4;

__device__ __forceinline__ int32_t claim_size(unsigned long long w) {
    const int32_t ph = w_phase(w);
    if (ph != kPhTri && ph != kPhScatter && ph != kPhTile) return 1;
    const uint32_t left = w_units(w) - min(w_units(w), w_next(w));
    return max(1, min(kMaxClaim, (int32_t)(left / kClaimDiv)));
}

__device__ __forceinline__ void publish(PSlotState& st, int32_t phase, int32_t n_units) {
    __hip_atomic_store(&st.done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&st.word, pword(phase, n_units), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ void st_dev(T* p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Put the next item into slot st (one lane). Batch: the next entry of the
// item list. Serving: the next published entry of the feed, if any.
__device__ bool admit(const PLaunch& P, PSlotState& st) {
    int32_t item, job, sun;
    if (!P.serve) {
        const uint32_t ni = atomicAdd(&P.sched->next_item, 1u);
        if (ni >= P.sched->n_items) return false;
        const PItem it = P.items[ni];
        item = (int32_t)ni;
        job = it.job;
        sun = it.sun;
    } else {
        for (;;) {
            uint32_t cur = ld_dev(&P.sched->next_item);
            const uint32_t pub = ld_dev(&P.sched->pub_dev);
            if ((int32_t)(pub - cur) <= 0) return false;
            if (__hip_atomic_compare_exchange_strong(&P.sched->next_item, &cur, cur + 1, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                const unsigned long long e = __hip_atomic_load(P.feed + (cur % P.feed_cap), __ATOMIC_ACQUIRE,
                                                               __HIP_MEMORY_SCOPE_SYSTEM);
                item = (int32_t)(cur & 0x7FFFFFFFu);
                job = (int32_t)(e >> 32);
                sun = (int32_t)(e & 0xFFFFFFFFu);
                // the job's table entry and inputs were copied in by the host before it published
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
                break;
            }
        }
    }
    st_dev(&st.item, item);
    st_dev(&st.job, job);
    st_dev(&st.sun, sun);
    st_dev(&st.overflow, 0);
    st_dev(&st.n_list, 0);
    return true;
}

// The last unit of a phase moves its item on (thread 0 decides; the whole
// workgroup runs the energy sum of a finished job).
__device__ void advance(const PLaunch& P, PCtl& ctl, double* stage, int32_t slot, int32_t phase) {
    const int tid = threadIdx.x;
    PSlotState& st = P.state[slot];
    const int32_t item = ld_dev(&st.item);
    const int32_t job = ld_dev(&st.job);
    const PJob& J = P.jobs[job];
    const PSlotBufs& B = P.slots[slot];
    if (tid == 0) {
        bool item_done = false;
        ctl.job_last = 0;
        switch (phase) {
            case kPhSetup:
                if (B.view->valid) {
                    const int64_t total = J.sc.n_tri + (J.g.occluders ? 2 * (int64_t)J.g.n_mod : 0) + J.g.n_mod;
                    publish(st, kPhTri, (int32_t)((total + kTriPerUnit - 1) / kTriPerUnit));
                } else {
                    publish(st, kPhLoss, 1);
                }
                break;
            case kPhTri: publish(st, kPhScan, 1); break;
            case kPhScan:
                if (ld_dev(&st.overflow)) {
                    item_done = true;
                } else {
                    const int32_t items = min(ld_dev(&B.ctr->n_rec), P.rec_cap) + J.g.n_mod;
                    publish(st, kPhScatter, max(1, (items + kScatterPerUnit - 1) / kScatterPerUnit));
                }
                break;
            case kPhScatter:
                if (ld_dev(&B.ctr->overflow)) {
                    st_dev(&st.overflow, 1);
                    item_done = true;
                } else {
                    const int32_t nl = ld_dev(&st.n_list);
                    if (nl > 0) publish(st, kPhTile, nl);
                    else publish(st, kPhLoss, 1);
                }
                break;
            case kPhTile: publish(st, kPhLoss, 1); break;
            default: item_done = true; break;
        }
        if (item_done) {
            if (ld_dev(&st.overflow)) {
                if (!P.serve) {
                    const uint32_t q = atomicAdd(&P.sched->n_overflow, 1u);
                    P.overflow_items[q] = item;
                } else {
                    // serving: the host evaluates the suns marked so again (the job's tag,
                    // released after every item of the job, orders this store before it)
                    J.power[ld_dev(&st.sun)] = __builtin_nan("");
                }
                atomicAdd(reinterpret_cast<uint32_t*>(&P.job_overflow[job]), 1u);
            }
            const uint32_t jd =
                __hip_atomic_fetch_add(&P.job_done[job], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT) + 1;
            if (jd == J.done_target) {
                const bool clean = (uint32_t)ld_dev(&P.job_overflow[job]) == J.ovf_base;
                ctl.job_last = clean ? 1 : 2;
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");   // the job's powers come from every XCD
            }
            ctl.job = job;
            // the slot takes the next item
            if (admit(P, st)) {
                publish(st, kPhSetup, 1);
            } else {
                if (P.serve) atomicSub(reinterpret_cast<uint32_t*>(&P.sched->busy), 1u);
                publish(st, kPhIdle, 0);
            }
            if (!ctl.job_last && !P.serve)
                __hip_atomic_fetch_add(&P.sched->items_done, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    __syncthreads();
    if (ctl.job_last) {
        const PJob& JJ = P.jobs[ctl.job];
        if (ctl.job_last == 1) {
            // energy of the finished job: sum of power * dt in sun order, as the per-sun path sums it
            double e = 0.0, er = 0.0;
            for (int64_t t0 = 0; t0 < JJ.n_sun; t0 += 256) {
                const int64_t t = t0 + tid;
                if (t < JJ.n_sun) {
                    stage[tid] = JJ.power[t];
                    stage[256 + tid] = JJ.power_ref[t];
                    stage[512 + tid] = JJ.dt[t];
                }
                __syncthreads();
                if (tid == 0) {
                    const int64_t m = min((int64_t)256, JJ.n_sun - t0);
                    for (int64_t q = 0; q < m; q++) {
                        e += stage[q] * stage[512 + q];
                        er += stage[256 + q] * stage[512 + q];
                    }
                }
                __syncthreads();
            }
            if (tid == 0) {
                JJ.energy[0] = e;
                JJ.energy[1] = er;
            }
        }
        if (tid == 0) {
            if (P.serve)      // outputs written back, then the tag the host waits for
                __hip_atomic_store(P.report + ctl.job, JJ.seq | (ctl.job_last == 2 ? 0x80000000u : 0u),
                                   __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            else
                __hip_atomic_fetch_add(&P.sched->items_done, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
}

__global__ __launch_bounds__(256, 3) void k_persist(PLaunch P) {
    __shared__ __attribute__((aligned(16))) unsigned char raw[kPLdsBytes];
    __shared__ PCtl ctl;
    const int tid = threadIdx.x, lane = tid & 63;
    // the slots this workgroup serves: my, my + G, my + 2G, ...
    const int32_t G = P.groups > 1 ? P.groups : 1;
    const int32_t my = G > 1 ? xcc_id() % G : 0;
    const int32_t n_mine = my < P.n_slots ? (P.n_slots - my + G - 1) / G : 0;
    int32_t home = n_mine > 0 ? (int32_t)((blockIdx.x / (unsigned)G) % (unsigned)n_mine) : 0;
    unsigned long long seen_units = ~0ull;
    long long seen_at = 0, quiet_since = -1, polled_at = -(1ll << 40);
    int32_t backoff = 1;
    for (;;) {
        if (P.serve && tid == 0 && (int32_t)blockIdx.x < kPollers) {
            // serving: a few workgroups copy the host's published count and stop flag into
            // device memory, at most every kPollTicks; every other workgroup reads the copies
            const long long now = (long long)wall_clock64();
            if (now - polled_at >= kPollTicks) {
                polled_at = now;
                const uint32_t pub = __hip_atomic_load(P.feed_pub, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
                if ((int32_t)(pub - ld_dev(&P.sched->pub_dev)) > 0) atomicMax(&P.sched->pub_dev, pub);
                if (__hip_atomic_load(P.stop_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0u)
                    st_dev(&P.sched->stop_dev, 1u);
            }
        }
        if (tid < 64) {                                   // wave 0 looks for a unit
            int32_t got = -1, gj = 0, unit = 0, phase = 0, units = 0, count = 0;
            const bool aborted = __hip_atomic_load(&P.sched->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
            for (int32_t base = 0; base < n_mine && got < 0 && !aborted; base += 64) {
                const int32_t kk = base + lane;
                int32_t j = home + kk;
                if (j >= n_mine) j -= n_mine;
                const int32_t i = my + j * G;
                // the oldest item with an open unit first: few items per XCD at a time keep
                // their buffers in its L2, while phases of younger items fill the gaps
                int32_t key = INT32_MAX;
                int32_t want = 1;
                if (kk < n_mine) {                      // word and item loaded together: one trip to L2
                    const unsigned long long w =
                        __hip_atomic_load(&P.state[i].word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    const int32_t itm = ld_dev(&P.state[i].item);
                    if (w_open(w)) key = itm;
                    // while serving, the feed pollers take one unit at a time: a poller held
                    // in a long claim leaves new items unseen and slots empty
                    want = (P.serve && (int32_t)blockIdx.x < kPollers) ? 1 : claim_size(w);
                }
                for (int attempt = 0; attempt < 64 && got < 0; attempt++) {
                    int32_t kmin = key, l = lane;
                    for (int off = 32; off > 0; off >>= 1) {
                        const int32_t k2 = __shfl_xor(kmin, off, 64), l2 = __shfl_xor(l, off, 64);
                        if (k2 < kmin || (k2 == kmin && l2 < l)) {
                            kmin = k2;
                            l = l2;
                        }
                    }
                    if (kmin == INT32_MAX) break;
                    int32_t ok = 0, u = 0, ph = 0, nu = 0, cn = 0;
                    if (lane == l) {
                        key = INT32_MAX;
                        // the phase may have moved on since the word was read: the claim
                        // covers whatever units of the current phase the add returns
                        const unsigned long long o = __hip_atomic_fetch_add(
                            &P.state[i].word, (unsigned long long)want, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (w_open(o)) {
                            ok = 1;
                            u = (int32_t)w_next(o);
                            ph = w_phase(o);
                            nu = (int32_t)w_units(o);
                            cn = min(want, nu - u);
                        }
                    }
                    ok = __shfl(ok, l, 64);
                    if (ok) {
                        got = __shfl(i, l, 64);
                        gj = __shfl(j, l, 64);
                        unit = __shfl(u, l, 64);
                        phase = __shfl(ph, l, 64);
                        units = __shfl(nu, l, 64);
                        count = __shfl(cn, l, 64);
                    }
                }
            }
            bool refilled = false;
            if (got < 0 && !aborted && P.serve && n_mine > 0) {
                // serving: an idle slot of this XCD takes a newly published item
                const uint32_t pub = ld_dev(&P.sched->pub_dev);
                if ((int32_t)(pub - ld_dev(&P.sched->next_item)) > 0) {
                    for (int32_t base = 0; base < n_mine && !refilled; base += 64) {
                        const int32_t kk = base + lane;
                        const int32_t i = my + kk * G;
                        unsigned long long w = 0;
                        bool idle = false;
                        if (kk < n_mine) {
                            w = __hip_atomic_load(&P.state[i].word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            idle = w_phase(w) == kPhIdle;
                        }
                        const unsigned long long m = __ballot(idle);
                        if (m != 0ull) {
                            const int l = __ffsll((long long)m) - 1;
                            if (lane == l) {
                                unsigned long long exp = w;
                                if (__hip_atomic_compare_exchange_strong(&P.state[i].word, &exp, pword(kPhAdmit, 0),
                                                                         __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                                         __HIP_MEMORY_SCOPE_AGENT)) {
                                    if (admit(P, P.state[i])) {
                                        atomicAdd(reinterpret_cast<uint32_t*>(&P.sched->busy), 1u);
                                        publish(P.state[i], kPhSetup, 1);
                                    } else {
                                        publish(P.state[i], kPhIdle, 0);
                                    }
                                }
                            }
                            refilled = true;
                        }
                    }
                }
            }
            if (got >= 0) {
                home = gj;
                backoff = 1;
            }
            if (lane == 0) {
                ctl.slot = got;
                ctl.unit = unit;
                ctl.phase = phase;
                ctl.units = units;
                ctl.count = count;
                ctl.stop = 0;
            }
            if (got >= 0) {
                if (lane == 0) acquire_unit(G);                // see what the unit's inputs' writers released
            } else if (!refilled) {
                bool stop = aborted, quiet = false;
                if (!stop && !P.serve) {
                    stop = __hip_atomic_load(&P.sched->items_done, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >=
                           P.sched->n_items;
                } else if (!stop) {
                    // serving: quiet when no slot holds an item and nothing waits in the feed
                    quiet = ld_dev(&P.sched->busy) <= 0 &&
                            (int32_t)(ld_dev(&P.sched->pub_dev) - ld_dev(&P.sched->next_item)) <= 0;
                }
                if (lane == 0) {
                    const long long now = (long long)wall_clock64();
                    if (!stop && quiet) {
                        if (quiet_since < 0) quiet_since = now;
                        if (ld_dev(&P.sched->stop_dev) != 0u || now - quiet_since > P.idle_ticks) stop = true;
                    } else if (!stop) {
                        quiet_since = -1;
                        const unsigned long long u =
                            __hip_atomic_load(&P.sched->units, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        if (u != seen_units) {
                            seen_units = u;
                            seen_at = now;
                        } else if (now - seen_at > P.stall_ticks) {
                            __hip_atomic_store(&P.sched->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            stop = true;
                        }
                    }
                    if (!stop)
                        for (int32_t q = 0; q < backoff; q++) __builtin_amdgcn_s_sleep(8);
                    ctl.stop = stop ? 1 : 0;
                }
                if (backoff < 32) backoff *= 2;
            }
        }
        __syncthreads();
        const int32_t slot = ctl.slot, unit = ctl.unit, phase = ctl.phase, count = ctl.count;
        if (slot < 0) {
            const int32_t stop = ctl.stop;
            __syncthreads();
            if (stop) break;
            continue;
        }
        {
            PSlotState& st = P.state[slot];
            const PItem it{ld_dev(&st.job), ld_dev(&st.sun)};
            const PJob& J = P.jobs[it.job];
            const PSlotBufs& B = P.slots[slot];
            const BinBuffers bb = slot_bins(P, J, B);
            switch (phase) {
                case kPhSetup: unit_setup(raw, J, it, B); break;
                case kPhTri:
                    for (int32_t q = 0; q < count; q++) {
                        if (q) __syncthreads();
                        unit_tri(raw, J, it, B, bb, unit + q);
                    }
                    break;
                case kPhScan: unit_scan(raw, P, J, B, bb, st); break;
                case kPhScatter:
                    for (int32_t q = 0; q < count; q++) {
                        if (q) __syncthreads();
                        unit_scatter(raw, J, B, bb, unit + q, ctl.units);
                    }
                    break;
                case kPhTile:
                    for (int32_t q = 0; q < count; q++) {
                        if (q) __syncthreads();
                        unit_tile(raw, J, it, B, bb, unit + q);
                    }
                    break;
                default: unit_loss(raw, J, it, B); break;
            }
        }
        // this unit's writes, before it counts as done: complete in the XCD's L2 when the
        // slot's readers share it, else (and for the powers the energy sum reads from
        // every XCD) written back to memory; while serving, the host's copy engine reads
        // a job's counts and powers as soon as its tag is set, so the last unit of every
        // item writes its XCD's dirty lines back for the host too
        if (P.serve && phase == kPhLoss)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
        else if (G > 1 && phase != kPhLoss)
            __builtin_amdgcn_s_waitcnt(kWaitVmem);
        else
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (tid == 0) {
            __hip_atomic_fetch_add(&P.sched->units, (unsigned long long)count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t d = __hip_atomic_fetch_add(&P.state[slot].done, (uint32_t)count, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT) + (uint32_t)count;
            ctl.finish = d == (uint32_t)ctl.units ? 1 : 0;
            if (ctl.finish) acquire_unit(G);                   // the other units of the phase
        }
        __syncthreads();
        if (ctl.finish) advance(P, ctl, reinterpret_cast<double*>(raw), slot, phase);
        __syncthreads();
    }
}

// Which XCD ids the workgroups of a launch run on (bit x of mask: XCD x).
__global__ void k_xcc_probe(uint32_t* mask) {
    if (threadIdx.x == 0) atomicOr(mask, 1u << (xcc_id() & 31));
}

inline unsigned grid_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
int32_t bounds_partials(int64_t n_points) {
    int64_t b = (n_points + 255) / 256;
    return (int32_t)(b < 1 ? 1 : (b > 1024 ? 1024 : b));
}

hipError_t launch_bounds(const SceneDev& sc, const GenDev& g, double* partial, int32_t n_part,
                         double* sphere, hipStream_t st) {
    hipLaunchKernelGGL(k_bounds_partial, dim3(n_part), dim3(256), 0, st, sc, g, partial);
    hipLaunchKernelGGL(k_bounds_final, dim3(1), dim3(64), 0, st, (const double*)partial, n_part, sphere);
    return hipGetLastError();
}

hipError_t launch_sample_tables(double* fu, double* fv, int32_t k, int32_t n_cu, int32_t n_cv,
                                hipStream_t st) {
    int32_t n = k * (n_cu > n_cv ? n_cu : n_cv);
    hipLaunchKernelGGL(k_sample_tables, dim3(grid_for(n, 256)), dim3(256), 0, st, fu, fv, k, n_cu, n_cv);
    return hipGetLastError();
}

hipError_t launch_setup(const double* sun, int64_t n_sun, const double* dni, const GenDev& g,
                        const double* sphere, int32_t n, View* views, double* beam, int32_t* bias,
                        const TileGrid& tg, uint32_t* tmask, hipStream_t st) {
    if (n_sun <= 0) return hipSuccess;
    if (tmask && tg.words > kMaxMaskWords) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_setup, dim3((unsigned)n_sun), dim3(256), 0, st, sun, dni, g, sphere, n, views,
                       beam, bias, tg, tmask);
    return hipGetLastError();
}

hipError_t launch_pose(const double* sun, int64_t n_sun, const Module* rest, int32_t n_mod, const TrackerDev* trk,
                       const int32_t* mod_trk, Module* posed, hipStream_t st) {
    const int64_t total = n_sun * n_mod;
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pose, dim3(grid_for(total, 256)), dim3(256), 0, st, sun, n_sun, rest, n_mod, trk, mod_trk,
                       posed);
    return hipGetLastError();
}

hipError_t launch_box_sphere(const double lo[3], const double hi[3], double* sphere, hipStream_t st) {
    hipLaunchKernelGGL(k_box_sphere, dim3(1), dim3(64), 0, st, lo[0], lo[1], lo[2], hi[0], hi[1], hi[2], sphere);
    return hipGetLastError();
}

hipError_t launch_tri_setup_group(const SunGroup* grp, int32_t n_sun, const View* views, const SceneDev& sc,
                                  const GenDev& g, const int32_t* bias, int32_t n, SunCounters* ctr, hipStream_t st) {
    const int64_t total = sc.n_tri + (g.occluders ? 2 * (int64_t)g.n_mod : 0) + g.n_mod;
    if (total == 0 || n_sun <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tri_setup_g, dim3(grid_for(total, 256), (unsigned)n_sun), dim3(256),
                       5 * sizeof(unsigned long long), st, grp, views, sc, bias, n, ctr);
    return hipGetLastError();
}

hipError_t launch_pair_count_group(const SunGroup* grp, int32_t grid, hipStream_t st) {
    hipLaunchKernelGGL(k_pair_count_g, dim3((unsigned)grid), dim3(256), 0, st, grp);
    return hipGetLastError();
}

hipError_t launch_pair_scatter_group(const SunGroup* grp, int32_t grid, hipStream_t st) {
    hipLaunchKernelGGL(k_pair_scatter_g, dim3((unsigned)grid), dim3(256), 0, st, grp);
    return hipGetLastError();
}

hipError_t launch_bin_scan_group(const SunGroup* grp, int32_t n_sun, int32_t n_tiles, hipStream_t st) {
    if (n_sun <= 0) return hipSuccess;
    if (n_tiles <= 512 * 8)
        hipLaunchKernelGGL((k_bin_scan_g<512, 8>), dim3((unsigned)n_sun), dim3(512), 0, st, grp, n_tiles);
    else if (n_tiles <= 512 * 32)
        hipLaunchKernelGGL((k_bin_scan_g<512, 32>), dim3((unsigned)n_sun), dim3(512), 0, st, grp, n_tiles);
    else
        hipLaunchKernelGGL((k_bin_scan_g<512, 8>), dim3((unsigned)n_sun), dim3(512), 0, st, grp, n_tiles);
    return hipGetLastError();
}

template <int TS, int CAP>
static hipError_t tile_go_group(const SunGroup* grp, int32_t n_sun, bool listed, int32_t n_tiles, const View* views,
                                const SunCounters* ctr, int32_t n, const int32_t* bias, const double* fu,
                                const double* fv, int32_t k, int32_t n_cu, int32_t cap_per_cu, hipStream_t st) {
    dim3 grid((unsigned)n_tiles, (unsigned)n_sun);
    if (listed) {
        static int per_cu = 0;                 // the same code object on every device of one architecture
        if (per_cu == 0) {
            int nb = 0;
            hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_tile_g<TS, CAP>, 256, 0);
            if (e != hipSuccess) return e;
            per_cu = nb > 0 ? nb : 1;
        }
        const int32_t use = cap_per_cu > 0 ? std::min(cap_per_cu, per_cu) : per_cu;
        const int64_t most = 4 * (int64_t)n_tiles * n_sun;
        grid = dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(most, (int64_t)n_cu * use)));
    }
    hipLaunchKernelGGL((k_tile_g<TS, CAP>), grid, dim3(256), 0, st, grp, views, ctr, n, bias, fu, fv, k);
    return hipGetLastError();
}

hipError_t launch_raster_group(const SunGroup* grp, int32_t n_sun, bool listed, int32_t tile, int32_t n_tiles,
                               const View* views, const SunCounters* ctr, int32_t n, const int32_t* bias,
                               int32_t n_mod, const double* fu, const double* fv, int32_t k, int32_t n_cu,
                               int32_t cap_per_cu, hipStream_t st) {
    (void)n_mod;
    if (n_sun <= 0) return hipSuccess;
    switch (tile) {
        case 32: return tile_go_group<32, kCap32>(grp, n_sun, listed, n_tiles, views, ctr, n, bias, fu, fv, k, n_cu, cap_per_cu, st);
        case 64: return tile_go_group<64, kCap64>(grp, n_sun, listed, n_tiles, views, ctr, n, bias, fu, fv, k, n_cu, cap_per_cu, st);
        case 128: return tile_go_group<128, kCap128>(grp, n_sun, listed, n_tiles, views, ctr, n, bias, fu, fv, k, n_cu, cap_per_cu, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_sample_test(int64_t s, const View* views, const GenDev& g, const double* beam,
                              const int32_t* bias, const double* fu, const double* fv, int32_t k,
                              const uint32_t* map, int32_t n, uint32_t* counts, uint32_t* bits,
                              hipStream_t st) {
    int64_t cells = (int64_t)g.n_mod * g.n_cu * g.n_cv;
    hipLaunchKernelGGL(k_sample_test, dim3(grid_for(cells, 4)), dim3(256), 0, st, s, views, g, beam, bias,
                       fu, fv, k, map, n, counts, bits);
    return hipGetLastError();
}

hipError_t launch_loss(int64_t s0, int64_t s1, const double* sun, const double* beam, const uint32_t* counts,
                       const double* d_poa, const GenDev& g, int32_t k, double* power, double* power_ref,
                       const SunCounters* ctr, hipStream_t st) {
    if (s1 <= s0) return hipSuccess;
    hipLaunchKernelGGL(k_loss, dim3((unsigned)(s1 - s0)), dim3(256), 0, st, s0, sun, beam, counts, d_poa, g, k,
                       power, power_ref, ctr);
    return hipGetLastError();
}

hipError_t launch_svf(const Module* mods, int32_t cpm, int64_t n_cells, const double* dirs, int64_t n_dir,
                      const uint32_t* counts, int32_t k, double* svf, hipStream_t st) {
    if (n_cells <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_svf, dim3((unsigned)((n_cells + 255) / 256)), dim3(256), 0, st, mods, cpm, n_cells, dirs,
                       n_dir, counts, k, svf);
    return hipGetLastError();
}

hipError_t launch_energy(int64_t n_sun, const double* power, const double* power_ref, const double* dt,
                         double* energy, hipStream_t st) {
    hipLaunchKernelGGL(k_energy, dim3(1), dim3(256), 0, st, n_sun, power, power_ref, dt, energy);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t b = grid_for(n, 256);
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)(b > 4096 ? 4096 : b)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

hipError_t launch_xcc_probe(uint32_t* mask, int32_t grid, hipStream_t st) {
    hipLaunchKernelGGL(k_xcc_probe, dim3((unsigned)grid), dim3(64), 0, st, mask);
    return hipGetLastError();
}

hipError_t persist_blocks_per_cu(int32_t* blocks) {
    int nb = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persist, 256, 0);
    *blocks = nb;
    return e;
}

hipError_t launch_persist(const PLaunch& P, int32_t grid, hipStream_t st) {
    if (grid <= 0 || P.n_slots <= 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_persist, dim3((unsigned)grid), dim3(256), 0, st, P);
    return hipGetLastError();
}

}  // namespace pv3d
