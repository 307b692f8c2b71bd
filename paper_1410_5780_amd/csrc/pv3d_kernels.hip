// HIP kernels of libpv3d for gfx950 (MI355X): the per-sun shadow-map path of
// arXiv:1410.5780, Sec. 2 Steps 3-4.
//
// Per sun position:
//   setup       one workgroup per sun: image basis, window over the module
//               corners, depth range, per-module beam and depth bias
//   tri_setup   one thread per triangle: FP64 light-space transform, culling,
//               guard-band clip, 1/256-texel snap, fixed-point edge and depth
//               planes, tile counts
//   bin_scan    exclusive scan of the tile counts (one workgroup)
//   bin_scatter one thread per set-up triangle: triangle ids into tile bins
//   raster      one workgroup per tile: depth tile in LDS, nearest depth by
//               ds_min_u32, 8x8-pixel stamps per wave, coalesced tile store
//   sample_test one wave per cell: FP64 affine map of the k x k sub-cell
//               samples, depth check against the picture, ballot + popcount
//   loss        one workgroup per sun: substring capacities, ideal bypass
//               string power, strings summed in order
//   energy      sum of power * dt in sun order
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

// ---------------------------------------------------------------------------
// generator preparation
// ---------------------------------------------------------------------------
__global__ void k_module_normals(Module* mods, int32_t n_mod) {
    int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_mod) return;
    d3 c = cross(ld3(mods[i].u), ld3(mods[i].v));
    double l = sqrt(dot(c, c));
    mods[i].n[0] = c.x / l;
    mods[i].n[1] = c.y / l;
    mods[i].n[2] = c.z / l;
}

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
// per-sun view and module terms
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_setup(const double* sun, const double* dni, GenDev g,
                                               const double* sphere, int32_t n, View* views,
                                               double* beam, int32_t* bias) {
    __shared__ double red[5][256];
    __shared__ int any_front;
    __shared__ View sv;
    const int64_t s = blockIdx.x;
    const int tid = threadIdx.x;
    const d3 sn = ld3(sun + 3 * s);
    const bool up = sn.z > 0.0;
    if (tid == 0) any_front = 0;
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
        views[s] = V;
    }
    __syncthreads();
    const double dn = dni[s];
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
        beam[s * g.n_mod + m] = bm;
        bias[s * g.n_mod + m] = bi;
    }
}

// ---------------------------------------------------------------------------
// triangle set-up and binning
// ---------------------------------------------------------------------------
__device__ __forceinline__ d3 to_light(const View& V, d3 p) {
    return d3{(dot(p, ld3(V.e1)) - V.ox) * V.itx, (dot(p, ld3(V.e2)) - V.oy) * V.ity,
              (dot(p, ld3(V.d)) - V.znear) * V.izd};
}

// Snap, orient and set up one light-space triangle; append it to the records
// and count it into the tiles it touches.
__device__ void emit_triangle(const d3 t[3], int32_t n, const BinBuffers& bb, SunCounters* ctr) {
    int64_t X[3], Y[3];
    double Z[3];
    const double tv[3][3] = {{t[0].x, t[0].y, t[0].z}, {t[1].x, t[1].y, t[1].z}, {t[2].x, t[2].y, t[2].z}};
    for (int q = 0; q < 3; q++) {
        X[q] = (int64_t)floor(tv[q][0] * 256.0 + 0.5);
        Y[q] = (int64_t)floor(tv[q][1] * 256.0 + 0.5);
        Z[q] = tv[q][2];
    }
    int64_t A = (X[1] - X[0]) * (Y[2] - Y[0]) - (X[2] - X[0]) * (Y[1] - Y[0]);
    if (A == 0) return;
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
    if (ilo > ihi || jlo > jhi) return;

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
        return;
    }
    bb.rec[idx] = r;
    const int32_t T = bb.tile;
    int32_t tx0 = (int32_t)ilo / T, tx1 = (int32_t)ihi / T, ty0 = (int32_t)jlo / T, ty1 = (int32_t)jhi / T;
    int32_t nt = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
    if (nt > bb.large_tiles) {
        int32_t li = atomicAdd(&ctr->n_large, 1);
        bb.large[li] = idx;
    } else {
        for (int32_t ty = ty0; ty <= ty1; ty++)
            for (int32_t tx = tx0; tx <= tx1; tx++) atomicAdd(&bb.tile_count[ty * bb.ntx + tx], 1);
    }
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

__device__ __noinline__ void clip_and_emit(const d3 t[3], int32_t n, const BinBuffers& bb, SunCounters* ctr) {
    d3 a[8], b[8];
    a[0] = t[0]; a[1] = t[1]; a[2] = t[2];
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
        emit_triangle(f, n, bb, ctr);
    }
}

__global__ __launch_bounds__(256) void k_tri_setup(int64_t s, const View* views, SceneDev sc, GenDev g,
                                                   int32_t n, BinBuffers bb, SunCounters* ctr) {
    const View& V = views[s];
    if (!V.valid) return;
    const int64_t total = sc.n_tri + (g.occluders ? 2 * (int64_t)g.n_mod : 0);
    const int64_t t = blockIdx.x * 256ll + threadIdx.x;
    if (t >= total) return;
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
    if (zmin > (double)kDepthMax) return;
    double xmin = fmin(l[0].x, fmin(l[1].x, l[2].x)), xmax = fmax(l[0].x, fmax(l[1].x, l[2].x));
    double ymin = fmin(l[0].y, fmin(l[1].y, l[2].y)), ymax = fmax(l[0].y, fmax(l[1].y, l[2].y));
    if (xmax < 0.0 || xmin >= (double)n || ymax < 0.0 || ymin >= (double)n) return;
    bool big = false;
    for (int q = 0; q < 3; q++)
        if (fabs(l[q].x) >= kGuard || fabs(l[q].y) >= kGuard) big = true;
    if (big) clip_and_emit(l, n, bb, ctr);
    else emit_triangle(l, n, bb, ctr);
}

__global__ __launch_bounds__(1024) void k_bin_scan(int32_t n_tiles, BinBuffers bb) {
    __shared__ int32_t part[1024];
    const int tid = threadIdx.x;
    const int32_t per = (n_tiles + 1023) / 1024;
    const int32_t b0 = min(tid * per, n_tiles), b1 = min(b0 + per, n_tiles);
    int32_t sum = 0;
    for (int32_t i = b0; i < b1; i++) sum += bb.tile_count[i];
    part[tid] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {     // inclusive Hillis-Steele scan
        int32_t v = tid >= off ? part[tid - off] : 0;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    int32_t run = part[tid] - sum;
    for (int32_t i = b0; i < b1; i++) {
        int32_t c = bb.tile_count[i];
        bb.tile_start[i] = run;
        bb.tile_cursor[i] = run;
        bb.tile_count[i] = 0;
        run += c;
    }
    if (tid == 1023) bb.tile_start[n_tiles] = part[1023];
}

__global__ __launch_bounds__(256) void k_bin_scatter(int64_t s, BinBuffers bb, SunCounters* ctr) {
    const int32_t n_rec = min(ctr[s].n_rec, bb.rec_cap);
    const int32_t idx = blockIdx.x * 256 + threadIdx.x;
    if (idx >= n_rec) return;
    const TriRec& r = bb.rec[idx];
    const int32_t T = bb.tile;
    int32_t tx0 = r.ilo / T, tx1 = r.ihi / T, ty0 = r.jlo / T, ty1 = r.jhi / T;
    if ((tx1 - tx0 + 1) * (ty1 - ty0 + 1) > bb.large_tiles) return;
    for (int32_t ty = ty0; ty <= ty1; ty++)
        for (int32_t tx = tx0; tx <= tx1; tx++) {
            int32_t pos = atomicAdd(&bb.tile_cursor[ty * bb.ntx + tx], 1);
            if (pos < bb.bin_cap) bb.bins[pos] = idx;
            else atomicOr(&ctr[s].overflow, 1);
        }
}

// ---------------------------------------------------------------------------
// raster: one workgroup per tile, nearest depth wins (Fig. 3)
// ---------------------------------------------------------------------------
template <int TS>
__global__ __launch_bounds__(256) void k_raster(int64_t s, const View* views, BinBuffers bb,
                                                const SunCounters* ctr, int32_t n, uint32_t* map) {
    constexpr int PITCH = TS + 8;                 // 8x8 stamp rows land in distinct banks
    __shared__ uint32_t zt[TS * PITCH];
    __shared__ int32_t next;
    const int tid = threadIdx.x, lane = tid & 63;
    const int32_t tile = blockIdx.x;
    const int32_t x0 = (tile % bb.ntx) * TS, y0 = (tile / bb.ntx) * TS;
    for (int q = tid; q < TS * PITCH; q += 256) zt[q] = kDepthMax;
    if (tid == 0) next = 0;
    __syncthreads();
    if (views[s].valid) {
        const int32_t n_large = ctr[s].n_large;
        const int32_t bs = min(bb.tile_start[tile], bb.bin_cap);
        const int32_t be = min(bb.tile_start[tile + 1], bb.bin_cap);
        const int32_t total = n_large + (be - bs);
        const int lx = lane & 7, ly = lane >> 3;
        for (;;) {
            int32_t got = 0;
            if (lane == 0) got = atomicAdd(&next, 1);
            const int32_t item = __builtin_amdgcn_readfirstlane(got);
            if (item >= total) break;
            const int32_t rid = __builtin_amdgcn_readfirstlane(item < n_large ? bb.large[item]
                                                                             : bb.bins[bs + item - n_large]);
            const TriRec& R = bb.rec[rid];
            const int32_t ilo = max((int32_t)R.ilo, x0), ihi = min((int32_t)R.ihi, x0 + TS - 1);
            const int32_t jlo = max((int32_t)R.jlo, y0), jhi = min((int32_t)R.jhi, y0 + TS - 1);
            if (ilo > ihi || jlo > jhi) continue;
            for (int32_t sy = (jlo - y0) & ~7; sy <= jhi - y0; sy += 8)
                for (int32_t sx = (ilo - x0) & ~7; sx <= ihi - x0; sx += 8) {
                    const int32_t px = x0 + sx + lx, py = y0 + sy + ly;
                    const int64_t E0 = R.e0[0] + ((int64_t)R.a[0] * px + (int64_t)R.b[0] * py) * 256;
                    const int64_t E1 = R.e0[1] + ((int64_t)R.a[1] * px + (int64_t)R.b[1] * py) * 256;
                    const int64_t E2 = R.e0[2] + ((int64_t)R.a[2] * px + (int64_t)R.b[2] * py) * 256;
                    if ((E0 | E1 | E2) >= 0) {
                        const int64_t z = R.z0 + (int64_t)px * R.gx + (int64_t)py * R.gy;
                        const int64_t zq = z >> 16;
                        const uint32_t D = zq < 0 ? 0u : (zq > (int64_t)kDepthMax ? kDepthMax : (uint32_t)zq);
                        atomicMin(&zt[(sy + ly) * PITCH + sx + lx], D);
                    }
                }
        }
    }
    __syncthreads();
    // coalesced tile store
    if ((n & 3) == 0) {
        for (int q = tid; q < TS * TS / 4; q += 256) {
            const int r = q / (TS / 4), c = (q % (TS / 4)) * 4;
            const int32_t py = y0 + r, px = x0 + c;
            if (py < n && px < n) {
                uint4 v;
                v.x = zt[r * PITCH + c]; v.y = zt[r * PITCH + c + 1];
                v.z = zt[r * PITCH + c + 2]; v.w = zt[r * PITCH + c + 3];
                *reinterpret_cast<uint4*>(map + (int64_t)py * n + px) = v;
            }
        }
    } else {
        for (int q = tid; q < TS * TS; q += 256) {
            const int r = q / TS, c = q % TS;
            const int32_t py = y0 + r, px = x0 + c;
            if (py < n && px < n) map[(int64_t)py * n + px] = zt[r * PITCH + c];
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

__global__ __launch_bounds__(256) void k_loss(const double* sun, const double* beam, const uint32_t* counts,
                                              const double* d_poa, GenDev g, int32_t k, double* power,
                                              double* power_ref) {
    __shared__ double cap[kMaxSubPerString];
    __shared__ double red[256];
    const int64_t s = blockIdx.x;
    const int tid = threadIdx.x;
    if (!(sun[3 * s + 2] > 0.0)) {
        if (tid == 0) { power[s] = 0.0; power_ref[s] = 0.0; }
        return;
    }
    const int32_t cpm = g.n_cu * g.n_cv;
    const int64_t n_cells = (int64_t)g.n_mod * cpm;
    const double kk = (double)(k * k);
    const double dp = d_poa[s];
    double tot[2] = {0.0, 0.0};
    for (int32_t st = 0; st < g.n_str; st++) {
        const int32_t m0 = g.str_start[st], m1 = g.str_start[st + 1];
        const int32_t nsub = (m1 - m0) * g.n_sub;
        for (int pass = 0; pass < 2; pass++) {
            for (int32_t q = tid; q < nsub; q += 256) {
                const int32_t m = g.str_mods[m0 + q / g.n_sub], sq = q % g.n_sub;
                const double bm = beam[s * g.n_mod + m];
                double cmin = INFINITY;
                for (int32_t c = 0; c < cpm; c++) {
                    if (g.cell_sub[c] != sq) continue;
                    const uint32_t sh = pass == 0 ? counts[s * n_cells + (int64_t)m * cpm + c] : 0u;
                    const double f = (double)sh / kk;
                    cmin = fmin(cmin, bm * (1.0 - f) + dp);
                }
                cap[q] = cmin;
            }
            __syncthreads();
            double best = 0.0;
            for (int32_t q = tid; q < nsub; q += 256) {
                const double v = cap[q];
                int32_t cnt = 0;
                for (int32_t r = 0; r < nsub; r++) cnt += cap[r] >= v ? 1 : 0;
                best = fmax(best, (double)cnt * v);
            }
            red[tid] = best;
            __syncthreads();
            for (int w = 128; w > 0; w >>= 1) {
                if (tid < w) red[tid] = fmax(red[tid], red[tid + w]);
                __syncthreads();
            }
            if (tid == 0) tot[pass] += red[0];
            __syncthreads();
        }
    }
    if (tid == 0) {
        power[s] = tot[0];
        power_ref[s] = tot[1];
    }
}

__global__ void k_energy(int64_t n_sun, const double* power, const double* power_ref, const double* dt,
                         double* energy) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double e = 0.0, er = 0.0;
    for (int64_t t = 0; t < n_sun; t++) {
        e += power[t] * dt[t];
        er += power_ref[t] * dt[t];
    }
    energy[0] = e;
    energy[1] = er;
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
    for (int64_t i = blockIdx.x * 256ll + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = v;
}

inline unsigned grid_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

// ---------------------------------------------------------------------------
// launch wrappers
// ---------------------------------------------------------------------------
hipError_t launch_module_normals(Module* mods, int32_t n_mod, hipStream_t st) {
    hipLaunchKernelGGL(k_module_normals, dim3(grid_for(n_mod, 256)), dim3(256), 0, st, mods, n_mod);
    return hipGetLastError();
}

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
                        hipStream_t st) {
    if (n_sun <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_setup, dim3((unsigned)n_sun), dim3(256), 0, st, sun, dni, g, sphere, n, views,
                       beam, bias);
    return hipGetLastError();
}

hipError_t launch_tri_setup(int64_t s, const View* views, const SceneDev& sc, const GenDev& g, int32_t n,
                            const BinBuffers& bb, SunCounters* ctr, hipStream_t st) {
    int64_t total = sc.n_tri + (g.occluders ? 2 * (int64_t)g.n_mod : 0);
    if (total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_tri_setup, dim3(grid_for(total, 256)), dim3(256), 0, st, s, views, sc, g, n, bb,
                       ctr + s);
    return hipGetLastError();
}

hipError_t launch_bin_scan(int32_t n_tiles, const BinBuffers& bb, hipStream_t st) {
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, st, n_tiles, bb);
    return hipGetLastError();
}

hipError_t launch_bin_scatter(int64_t s, const BinBuffers& bb, int32_t n_tiles, SunCounters* ctr,
                              hipStream_t st) {
    (void)n_tiles;
    hipLaunchKernelGGL(k_bin_scatter, dim3(grid_for(bb.rec_cap, 256)), dim3(256), 0, st, s, bb, ctr);
    return hipGetLastError();
}

hipError_t launch_raster(int64_t s, const View* views, const BinBuffers& bb, const SunCounters* ctr,
                         int32_t n, uint32_t* map, hipStream_t st) {
    int32_t nt = (n + bb.tile - 1) / bb.tile;
    dim3 grid((unsigned)(nt * nt));
    switch (bb.tile) {
        case 32: hipLaunchKernelGGL(k_raster<32>, grid, dim3(256), 0, st, s, views, bb, ctr, n, map); break;
        case 64: hipLaunchKernelGGL(k_raster<64>, grid, dim3(256), 0, st, s, views, bb, ctr, n, map); break;
        case 128: hipLaunchKernelGGL(k_raster<128>, grid, dim3(256), 0, st, s, views, bb, ctr, n, map); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
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

hipError_t launch_loss(int64_t n_sun, const double* sun, const double* beam, const uint32_t* counts,
                       const double* d_poa, const GenDev& g, int32_t k, double* power, double* power_ref,
                       hipStream_t st) {
    if (n_sun <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_loss, dim3((unsigned)n_sun), dim3(256), 0, st, sun, beam, counts, d_poa, g, k, power,
                       power_ref);
    return hipGetLastError();
}

hipError_t launch_energy(int64_t n_sun, const double* power, const double* power_ref, const double* dt,
                         double* energy, hipStream_t st) {
    hipLaunchKernelGGL(k_energy, dim3(1), dim3(64), 0, st, n_sun, power, power_ref, dt, energy);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    int64_t b = grid_for(n, 256);
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)(b > 4096 ? 4096 : b)), dim3(256), 0, st, p, v, n);
    return hipGetLastError();
}

}  // namespace pv3d
