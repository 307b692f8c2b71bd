/*
 * pv3d oracle: a plain, slow CPU reference of the shadow-map shading path of
 * Robledo, Leloux & Lorenzo, "3D simulation of complex shading affecting PV
 * systems taking benefit from the power of graphics cards developed for the
 * video game industry" (arXiv:1410.5780).
 *
 * TEST INFRASTRUCTURE ONLY. Nothing on the product path links, loads or calls
 * this file: only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark do. It shares no code, header or constant table with the HIP
 * library; both sides are written independently from the paper.
 *
 * What is computed (Sec. 2, Steps 3 and 4):
 *   for every sun position the scene is drawn with an orthographic view from
 *   the sun whose field of view is limited to the PV generator; a depth buffer
 *   keeps, per pixel, the depth of the surface nearest to the sun (Fig. 3);
 *   every point of interest on the generator is then depth-checked against
 *   that picture: it is lit when its depth matches the stored one and shaded
 *   when it lies farther from the sun (Step 3, Fig. 4). The generator is split
 *   into small areas per cell (Step 3, last paragraph). Shaded areas lose the
 *   direct component of the irradiance (Step 4), an electrical model turns the
 *   geometric shading into power, and the per-moment results are integrated
 *   over time (Step 4, last two paragraphs).
 *
 * The paper leaves the rasterizer's arithmetic, the depth precision, the
 * depth bias and the electrical model unspecified; the readings taken here
 * (24-bit depth, 8 sub-pixel bits, top-left fill rule, slope-scaled bias,
 * ideal bypass-diode model) are listed with the design notes. Everything is
 * evaluated in IEEE binary64 with no contraction (build with
 * -ffp-contract=off), every dot product as (ax*bx + ay*by) + az*bz.
 *
 * Trackers (Sec. 3.4): generators whose modules turn about a pivot to follow
 * the sun are evaluated with the modules posed anew for every sun (see the
 * tracker section below for the reading of the tracking law).
 *
 * Electrical model (Step 4): ideal bypass-diode strings by default, or the
 * single-diode cell model with bypass diodes and a maximum power point per
 * string (see its section below). Diffuse shading (Sec. 4): per-cell sky view
 * factors from fixed sky directions, each evaluated as a sun, scale each
 * cell's diffuse (see the sky view section below).
 *
 * Parallelism: sun positions are independent, so the driver runs one sun per
 * OpenMP thread; the work inside one sun is plain sequential loops.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_SUBPIX 8                   /* sub-pixel bits of snapped vertices */
#define OR_DMAX 16777215              /* 2^24 - 1: farthest representable depth */
#define OR_GUARD 2097152.0            /* 2^21 texels: clip square for huge triangles */

typedef struct { double x, y, z; } v3;

static v3 mk(double x, double y, double z) { v3 r; r.x = x; r.y = y; r.z = z; return r; }
static v3 add3(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3 sub3(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static double dot3(v3 a, v3 b) { return (a.x * b.x + a.y * b.y) + a.z * b.z; }
static v3 cross3(v3 a, v3 b) {
    return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static v3 ld3(const double* p) { return mk(p[0], p[1], p[2]); }

/* floor(a / 2^s) for signed a, written without relying on signed shifts */
static int64_t floor_div_pow2(int64_t a, int s) {
    int64_t q = ((int64_t)1) << s;
    if (a >= 0) return a / q;
    return -((-a + q - 1) / q);
}

/* ------------------------------------------------------------------------ */
/* inputs                                                                   */
/* ------------------------------------------------------------------------ */
typedef struct {
    const double* xyz; int64_t n_vert;
    const int32_t* tri; int64_t n_tri;
    const double* org; const double* eu; const double* ev; int64_t n_mod;
    int32_t n_cu, n_cv;
    const int32_t* cell_sub; int32_t n_sub;
    const int32_t* mod_string; int32_t n_string;
    int32_t occluders;            /* 1: each module is also drawn as two triangles */
    const double* diode;          /* single-diode cell parameters, or NULL: ideal strings */
    const double* svf;            /* [n_mod * n_cu * n_cv] share of the diffuse each cell gets, or NULL: all */
} or_problem;

typedef struct {
    v3 s, d, e1, e2;              /* sun, view direction (away from the sun), image axes */
    double ox, oy, itx, ity;      /* window origin and texels per metre */
    double znear, izd;            /* depth origin and depth units per metre */
    int32_t n;                    /* map is n x n */
    int32_t valid;                /* 0: nothing drawn (sun down or no front-lit module) */
} or_view;

static void module_corners(const or_problem* P, int64_t m, v3 c[4]) {
    v3 o = ld3(P->org + 3 * m), u = ld3(P->eu + 3 * m), v = ld3(P->ev + 3 * m);
    c[0] = o;
    c[1] = add3(o, u);
    c[2] = add3(add3(o, u), v);
    c[3] = add3(o, v);
}

/* Bounding sphere of everything drawn or tested: centre of the axis-aligned
 * box of all scene vertices and module corners, radius its half diagonal. */
static void scene_sphere(const or_problem* P, v3* centre, double* radius) {
    v3 lo = mk(INFINITY, INFINITY, INFINITY), hi = mk(-INFINITY, -INFINITY, -INFINITY);
    for (int64_t i = 0; i < P->n_vert + 4 * P->n_mod; i++) {
        v3 p;
        if (i < P->n_vert) {
            p = ld3(P->xyz + 3 * i);
        } else {
            v3 c[4];
            int64_t j = i - P->n_vert;
            module_corners(P, j / 4, c);
            p = c[j % 4];
        }
        lo.x = p.x < lo.x ? p.x : lo.x; hi.x = p.x > hi.x ? p.x : hi.x;
        lo.y = p.y < lo.y ? p.y : lo.y; hi.y = p.y > hi.y ? p.y : hi.y;
        lo.z = p.z < lo.z ? p.z : lo.z; hi.z = p.z > hi.z ? p.z : hi.z;
    }
    *centre = mk((lo.x + hi.x) * 0.5, (lo.y + hi.y) * 0.5, (lo.z + hi.z) * 0.5);
    v3 dg = sub3(hi, lo);
    *radius = 0.5 * sqrt(dot3(dg, dg));
}

static v3 unit_normal(const or_problem* P, int64_t m) {
    v3 n = cross3(ld3(P->eu + 3 * m), ld3(P->ev + 3 * m));
    double l = sqrt(dot3(n, n));
    return mk(n.x / l, n.y / l, n.z / l);
}

/* Orthographic view from the sun limited to the generator (Sec. 2, Step 3):
 * image axes e1, e2 orthogonal to the view direction d = -s; the window is the
 * bounding box of all module corners plus one texel of margin on each side,
 * with independent texel sizes along e1 and e2; depth runs from the near side
 * of the bounding sphere (0) to the generator's farthest corner (2^24 - 1). */
static void view_setup(const or_problem* P, v3 s, int32_t n, v3 centre, double radius, or_view* V) {
    memset(V, 0, sizeof(*V));
    V->n = n;
    V->s = s;
    if (!(s.z > 0.0)) return;                      /* below the horizon */
    int any_front = 0;
    for (int64_t m = 0; m < P->n_mod; m++)
        if (dot3(unit_normal(P, m), s) > 0.0) any_front = 1;
    if (!any_front) return;
    V->d = mk(-s.x, -s.y, -s.z);
    v3 a = fabs(V->d.z) < 0.9 ? mk(0.0, 0.0, 1.0) : mk(1.0, 0.0, 0.0);
    v3 w = cross3(a, V->d);
    double wl = sqrt(dot3(w, w));
    V->e1 = mk(w.x / wl, w.y / wl, w.z / wl);
    V->e2 = cross3(V->d, V->e1);
    double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY, zfar = -INFINITY;
    for (int64_t m = 0; m < P->n_mod; m++) {
        v3 c[4];
        module_corners(P, m, c);
        for (int q = 0; q < 4; q++) {
            double u = dot3(c[q], V->e1), v = dot3(c[q], V->e2), z = dot3(c[q], V->d);
            if (u < umin) umin = u;
            if (u > umax) umax = u;
            if (v < vmin) vmin = v;
            if (v > vmax) vmax = v;
            if (z > zfar) zfar = z;
        }
    }
    double su = umax - umin, sv = vmax - vmin;
    if (!(su > 0.0 && sv > 0.0)) return;
    V->itx = (double)(n - 2) / su;
    V->ity = (double)(n - 2) / sv;
    V->ox = umin - su / (double)(n - 2);
    V->oy = vmin - sv / (double)(n - 2);
    V->znear = dot3(centre, V->d) - radius;
    V->izd = (double)OR_DMAX / (zfar - V->znear);
    V->valid = 1;
}

static v3 to_light(const or_view* V, v3 p) {
    return mk((dot3(p, V->e1) - V->ox) * V->itx,
              (dot3(p, V->e2) - V->oy) * V->ity,
              (dot3(p, V->d) - V->znear) * V->izd);
}

/* ------------------------------------------------------------------------ */
/* raster into the depth picture (Fig. 3: the nearest depth per pixel wins)   */
/* ------------------------------------------------------------------------ */
/* One triangle with its corners already in light space (x, y in texels, z in
 * depth units). Pixel (i, j) is sampled at its centre. Vertices are snapped
 * to 1/256 texel; a centre is inside when all three edge functions are
 * positive, or zero on a top or left edge; the depth is a fixed-point plane
 * (16 fraction bits) anchored at one pixel per triangle. */
static void raster_snapped(const double t[3][3], int32_t n, uint32_t* map, uint32_t* cover) {
    int64_t X[3], Y[3];
    double Z[3];
    for (int q = 0; q < 3; q++) {
        X[q] = (int64_t)floor(t[q][0] * 256.0 + 0.5);
        Y[q] = (int64_t)floor(t[q][1] * 256.0 + 0.5);
        Z[q] = t[q][2];
    }
    int64_t A = (X[1] - X[0]) * (Y[2] - Y[0]) - (X[2] - X[0]) * (Y[1] - Y[0]);
    if (A == 0) return;
    if (A < 0) {                      /* make the winding counter-clockwise */
        int64_t tx = X[1]; X[1] = X[2]; X[2] = tx;
        int64_t ty = Y[1]; Y[1] = Y[2]; Y[2] = ty;
        double tz = Z[1]; Z[1] = Z[2]; Z[2] = tz;
        A = -A;
    }
    /* edges a -> b: v1 -> v2, v2 -> v0, v0 -> v1 */
    int ea[3] = {1, 2, 0}, eb[3] = {2, 0, 1};
    int topleft[3];
    for (int e = 0; e < 3; e++) {
        int64_t dx = X[eb[e]] - X[ea[e]], dy = Y[eb[e]] - Y[ea[e]];
        topleft[e] = (dy < 0) || (dy == 0 && dx < 0);
    }
    /* depth plane through the snapped corners */
    double Ad = (double)A / 65536.0;
    double dx1 = (double)(X[1] - X[0]) / 256.0, dy1 = (double)(Y[1] - Y[0]) / 256.0;
    double dx2 = (double)(X[2] - X[0]) / 256.0, dy2 = (double)(Y[2] - Y[0]) / 256.0;
    double dz1 = Z[1] - Z[0], dz2 = Z[2] - Z[0];
    double gx = (dz1 * dy2 - dz2 * dy1) / Ad;
    double gy = (dx1 * dz2 - dx2 * dz1) / Ad;
    const double GLIM = 1073741824.0;             /* 2^30 depth units per texel */
    if (gx > GLIM) gx = GLIM;
    if (gx < -GLIM) gx = -GLIM;
    if (gy > GLIM) gy = GLIM;
    if (gy < -GLIM) gy = -GLIM;
    int64_t xmin = X[0], xmax = X[0], ymin = Y[0], ymax = Y[0];
    for (int q = 1; q < 3; q++) {
        if (X[q] < xmin) xmin = X[q];
        if (X[q] > xmax) xmax = X[q];
        if (Y[q] < ymin) ymin = Y[q];
        if (Y[q] > ymax) ymax = Y[q];
    }
    int64_t i0 = floor_div_pow2(xmin, OR_SUBPIX), j0 = floor_div_pow2(ymin, OR_SUBPIX);
    if (i0 < 0) i0 = 0;
    if (i0 > n - 1) i0 = n - 1;
    if (j0 < 0) j0 = 0;
    if (j0 > n - 1) j0 = n - 1;
    double za = (Z[0] + gx * (((double)i0 + 0.5) - (double)X[0] / 256.0))
                + gy * (((double)j0 + 0.5) - (double)Y[0] / 256.0);
    const double ZLIM = 1099511627776.0;          /* 2^40 */
    if (za > ZLIM) za = ZLIM;
    if (za < -ZLIM) za = -ZLIM;
    int64_t gxf = (int64_t)floor(gx * 65536.0 + 0.5);
    int64_t gyf = (int64_t)floor(gy * 65536.0 + 0.5);
    int64_t zaf = (int64_t)floor(za * 65536.0 + 0.5);
    /* pixels whose centres can lie in the snapped bounding box */
    int64_t ilo = -floor_div_pow2(-(xmin - 128), OR_SUBPIX);   /* ceil((xmin-128)/256) */
    int64_t ihi = floor_div_pow2(xmax - 128, OR_SUBPIX);
    int64_t jlo = -floor_div_pow2(-(ymin - 128), OR_SUBPIX);
    int64_t jhi = floor_div_pow2(ymax - 128, OR_SUBPIX);
    if (ilo < 0) ilo = 0;
    if (jlo < 0) jlo = 0;
    if (ihi > n - 1) ihi = n - 1;
    if (jhi > n - 1) jhi = n - 1;
    for (int64_t j = jlo; j <= jhi; j++) {
        int64_t py = j * 256 + 128;
        for (int64_t i = ilo; i <= ihi; i++) {
            int64_t px = i * 256 + 128;
            int inside = 1;
            for (int e = 0; e < 3; e++) {
                int64_t xa = X[ea[e]], ya = Y[ea[e]], xb = X[eb[e]], yb = Y[eb[e]];
                int64_t E = (xb - xa) * (py - ya) - (yb - ya) * (px - xa);
                if (!(E > 0 || (E == 0 && topleft[e]))) { inside = 0; break; }
            }
            if (!inside) continue;
            int64_t D = floor_div_pow2(zaf + (i - i0) * gxf + (j - j0) * gyf, 16);
            if (D < 0) D = 0;
            if (D > OR_DMAX) D = OR_DMAX;
            if ((uint32_t)D < map[j * (int64_t)n + i]) map[j * (int64_t)n + i] = (uint32_t)D;
            if (cover) cover[j * (int64_t)n + i] += 1;
        }
    }
}

/* Sutherland-Hodgman against one side of the guard square; the clipped
 * coordinate is set exactly on the boundary, the other two interpolated. */
static int clip_side(double in[][3], int nin, double out[][3], int axis, double c, int keep_ge) {
    int m = 0;
    for (int q = 0; q < nin; q++) {
        double* p = in[q];
        double* r = in[(q + 1) % nin];
        int pin = keep_ge ? (p[axis] >= c) : (p[axis] <= c);
        int rin = keep_ge ? (r[axis] >= c) : (r[axis] <= c);
        if (pin) {
            out[m][0] = p[0]; out[m][1] = p[1]; out[m][2] = p[2];
            m++;
        }
        if (pin != rin) {
            double t = (c - p[axis]) / (r[axis] - p[axis]);
            for (int k = 0; k < 3; k++) out[m][k] = p[k] + (r[k] - p[k]) * t;
            out[m][axis] = c;
            m++;
        }
    }
    return m;
}

static void raster_light_triangle(const double t[3][3], int32_t n, uint32_t* map, uint32_t* cover) {
    double xmin = t[0][0], xmax = t[0][0], ymin = t[0][1], ymax = t[0][1], zmin = t[0][2];
    for (int q = 1; q < 3; q++) {
        if (t[q][0] < xmin) xmin = t[q][0];
        if (t[q][0] > xmax) xmax = t[q][0];
        if (t[q][1] < ymin) ymin = t[q][1];
        if (t[q][1] > ymax) ymax = t[q][1];
        if (t[q][2] < zmin) zmin = t[q][2];
    }
    if (zmin > (double)OR_DMAX) return;                      /* wholly behind the generator */
    if (xmax < 0.0 || xmin >= (double)n || ymax < 0.0 || ymin >= (double)n) return;
    int big = 0;
    for (int q = 0; q < 3; q++)
        if (fabs(t[q][0]) >= OR_GUARD || fabs(t[q][1]) >= OR_GUARD) big = 1;
    if (!big) {
        raster_snapped(t, n, map, cover);
        return;
    }
    double a[8][3], b[8][3];
    int m = 3;
    for (int q = 0; q < 3; q++) { a[q][0] = t[q][0]; a[q][1] = t[q][1]; a[q][2] = t[q][2]; }
    m = clip_side(a, m, b, 0, -OR_GUARD, 1);
    if (m < 3) return;
    m = clip_side(b, m, a, 0, OR_GUARD, 0);
    if (m < 3) return;
    m = clip_side(a, m, b, 1, -OR_GUARD, 1);
    if (m < 3) return;
    m = clip_side(b, m, a, 1, OR_GUARD, 0);
    if (m < 3) return;
    for (int q = 1; q + 1 < m; q++) {
        double f[3][3];
        for (int k = 0; k < 3; k++) { f[0][k] = a[0][k]; f[1][k] = a[q][k]; f[2][k] = a[q + 1][k]; }
        raster_snapped(f, n, map, cover);
    }
}

/* ------------------------------------------------------------------------ */
/* one sun position                                                         */
/* ------------------------------------------------------------------------ */
/* per-thread scratch: cap [n_mod * n_cu * n_cv] doubles, sub_len [n_mod * n_sub] */
typedef struct { double* cap; int32_t* sub_len; } or_scratch;

static int cmp_desc(const void* a, const void* b) {
    double x = *(const double*)a, y = *(const double*)b;
    return (x < y) - (x > y);
}

/* Ideal bypass-diode string: substrings in series, each either carries the
 * string current at unit voltage or is bypassed at zero voltage; the string
 * works at the current that maximises power, i.e. max_j j * I_(j) over the
 * substring capacities sorted in decreasing order. */
static double string_power(double* caps, int64_t n) {
    qsort(caps, (size_t)n, sizeof(double), cmp_desc);
    double best = 0.0;
    for (int64_t j = 0; j < n; j++) {
        double p = (double)(j + 1) * caps[j];
        if (p > best) best = p;
    }
    return best;
}

/* Generator power for one sun: cell irradiance is the beam on the module
 * minus its shaded share plus the diffuse; a substring carries at most the
 * irradiance of its weakest cell; strings add up. */
static double generator_power(const or_problem* P, const double* beam, const uint32_t* counts,
                              int32_t k, double d_poa, double* caps) {
    int64_t cpm = (int64_t)P->n_cu * P->n_cv;
    double total = 0.0;
    for (int32_t st = 0; st < P->n_string; st++) {
        int64_t nc = 0;
        for (int64_t m = 0; m < P->n_mod; m++) {
            if (P->mod_string[m] != st) continue;
            for (int32_t q = 0; q < P->n_sub; q++) {
                double cmin = INFINITY;
                for (int64_t c = 0; c < cpm; c++) {
                    if (P->cell_sub[c] != q) continue;
                    uint32_t sh = counts ? counts[m * cpm + c] : 0u;
                    double f = (double)sh / (double)(k * k);
                    double sky = counts && P->svf ? P->svf[m * cpm + c] : 1.0;   /* reference: whole sky */
                    double g = beam[m] * (1.0 - f) + d_poa * sky;
                    if (g < cmin) cmin = g;
                }
                caps[nc++] = cmin;
            }
        }
        total += string_power(caps, nc);
    }
    return total;
}

/* ------------------------------------------------------------------------ */
/* single-diode electrical model                                            */
/* ------------------------------------------------------------------------ */
/* Step 4 turns the geometric shading into power with a diode model of the
 * cells and a model of the system, neither given in the paper. Reading taken
 * for this model: every cell follows the five-parameter single-diode equation
 *   I = Iph - I0 (exp((V + I Rs) / a) - 1) - (V + I Rs) / Rsh,
 * with the photocurrent proportional to the cell's irradiance,
 * Iph = Isc_ref G / G_ref, at a fixed cell temperature (a = n k T / q given).
 * The cells of a substring are in series and its bypass diode holds the
 * substring's voltage at no less than -Vb; substrings are in series in a
 * string, and each string works at its own maximum power point.
 * Parameters: d[0] Isc_ref (A), d[1] G_ref (W/m^2), d[2] I0 (A), d[3] a (V),
 * d[4] Rs (ohm), d[5] Rsh (ohm), d[6] Vb (V). */
#define OR_MPP_GRID 64       /* current grid of the maximum power search */
#define OR_MPP_REFINE 40     /* golden-section steps around each grid maximum */

/* Voltage of one cell carrying current I at irradiance G. With x = V + I Rs
 * the equation reads f(x) = c - I0 exp(x / a) - x / Rsh = 0, c = Iph + I0 - I;
 * f falls and is concave, so Newton's method started at a point where f <= 0
 * goes down to the root without passing it. Such a start: x = Rsh c (there
 * f = -I0 exp(x/a) < 0), and when c >= I0 also x = a ln(c / I0) (there
 * f = -x / Rsh <= 0); the smaller of the two is taken. The iteration stops
 * when a step no longer lowers x. */
static double cell_voltage(const double* d, double G, double I) {
    double iph = d[0] * G / d[1];
    double c = iph + d[2] - I;
    double x = d[5] * c;
    if (c >= d[2]) {
        double xl = d[3] * log(c / d[2]);
        if (xl < x) x = xl;
    }
    for (int it = 0; it < 64; it++) {
        double e = exp(x / d[3]);
        double f = (c - d[2] * e) - x / d[5];
        double fp = -(d[2] / d[3]) * e - 1.0 / d[5];
        double xn = x - f / fp;
        if (!(xn < x)) break;
        x = xn;
    }
    return x - I * d[4];
}

/* String voltage at current I: g holds the irradiance of every cell of the
 * string, substring after substring; sub_len the number of cells of each of
 * its n_q substrings. */
static double string_voltage(const double* d, const double* g, const int32_t* sub_len, int64_t n_q, double I) {
    double v = 0.0;
    int64_t c = 0;
    for (int64_t q = 0; q < n_q; q++) {
        double vs = 0.0;
        for (int32_t i = 0; i < sub_len[q]; i++) vs += cell_voltage(d, g[c + i], I);
        c += sub_len[q];
        if (vs < -d[6]) vs = -d[6];
        v += vs;
    }
    return v;
}

static double string_p(const double* d, const double* g, const int32_t* sub_len, int64_t n_q, double I) {
    return I * string_voltage(d, g, sub_len, n_q, I);
}

/* Maximum power of one string over its currents [0, Imax], Imax the largest
 * photocurrent of its cells (above it every cell is reverse-biased). The
 * power is sampled at OR_MPP_GRID + 1 evenly spaced currents; around every
 * sample that is not below its neighbours, a golden-section search over the
 * two grid steps beside it refines the maximum. The largest value seen (and
 * at least 0) is the string's power. */
static double string_mpp(const double* d, const double* g, const int32_t* sub_len, int64_t n_q) {
    int64_t n_c = 0;
    for (int64_t q = 0; q < n_q; q++) n_c += sub_len[q];
    double imax = 0.0;
    for (int64_t c = 0; c < n_c; c++) {
        double iph = d[0] * g[c] / d[1];
        if (iph > imax) imax = iph;
    }
    if (!(imax > 0.0)) return 0.0;
    double p[OR_MPP_GRID + 1];
    for (int q = 0; q <= OR_MPP_GRID; q++)
        p[q] = string_p(d, g, sub_len, n_q, imax * (double)q / (double)OR_MPP_GRID);
    const double r = 0.6180339887498949;       /* (sqrt(5) - 1) / 2 */
    double best = 0.0;
    for (int q = 1; q <= OR_MPP_GRID; q++) {
        if (!(p[q] >= p[q - 1]) || (q < OR_MPP_GRID && !(p[q] >= p[q + 1]))) continue;
        if (p[q] > best) best = p[q];
        double lo = imax * (double)(q - 1) / (double)OR_MPP_GRID;
        double hi = imax * (double)(q < OR_MPP_GRID ? q + 1 : q) / (double)OR_MPP_GRID;
        double xc = hi - r * (hi - lo), xd = lo + r * (hi - lo);
        double fc = string_p(d, g, sub_len, n_q, xc), fd = string_p(d, g, sub_len, n_q, xd);
        if (fc > best) best = fc;
        if (fd > best) best = fd;
        for (int it = 0; it < OR_MPP_REFINE; it++) {
            if (fc >= fd) {
                hi = xd; xd = xc; fd = fc;
                xc = hi - r * (hi - lo);
                fc = string_p(d, g, sub_len, n_q, xc);
                if (fc > best) best = fc;
            } else {
                lo = xc; xc = xd; fc = fd;
                xd = lo + r * (hi - lo);
                fd = string_p(d, g, sub_len, n_q, xd);
                if (fd > best) best = fd;
            }
        }
    }
    return best;
}

/* Generator power for one sun with the single-diode model: per string, the
 * irradiance of each cell (beam on the module minus its shaded share, plus
 * the diffuse), substring by substring in module order, then the string's
 * maximum power; strings add up. g and sub_len are scratch of n_cells and
 * n_mod * n_sub entries. */
static double generator_power_diode(const or_problem* P, const double* beam, const uint32_t* counts,
                                    int32_t k, double d_poa, double* g, int32_t* sub_len) {
    int64_t cpm = (int64_t)P->n_cu * P->n_cv;
    double total = 0.0;
    for (int32_t st = 0; st < P->n_string; st++) {
        int64_t nq = 0, nc = 0;
        for (int64_t m = 0; m < P->n_mod; m++) {
            if (P->mod_string[m] != st) continue;
            for (int32_t q = 0; q < P->n_sub; q++) {
                int32_t len = 0;
                for (int64_t c = 0; c < cpm; c++) {
                    if (P->cell_sub[c] != q) continue;
                    uint32_t sh = counts ? counts[m * cpm + c] : 0u;
                    double f = (double)sh / (double)(k * k);
                    double sky = counts && P->svf ? P->svf[m * cpm + c] : 1.0;   /* reference: whole sky */
                    g[nc++] = beam[m] * (1.0 - f) + d_poa * sky;
                    len++;
                }
                sub_len[nq++] = len;
            }
        }
        total += string_mpp(P->diode, g, sub_len, nq);
    }
    return total;
}

typedef struct {
    uint32_t* counts;      /* [n_cells] */
    uint32_t* bits;        /* [n_cells][words] or NULL */
    uint32_t* map;         /* [n][n] working or exported depth picture */
    double power, power_ref;
    int64_t outside;       /* samples that fell outside the map (must stay 0) */
} or_sun_out;

static void eval_sun(const or_problem* P, v3 centre, double radius, const double* s_in, double dni,
                     double d_poa, int32_t n, int32_t k, or_sun_out* o, double* beam, int32_t* bias,
                     or_scratch* sc) {
    int64_t cpm = (int64_t)P->n_cu * P->n_cv;
    int64_t nn = (int64_t)n * n;
    int32_t words = (k * k + 31) / 32;
    for (int64_t c = 0; c < P->n_mod * cpm; c++) o->counts[c] = 0;
    if (o->bits) memset(o->bits, 0, sizeof(uint32_t) * (size_t)(P->n_mod * cpm * words));
    for (int64_t p = 0; p < nn; p++) o->map[p] = OR_DMAX;
    o->outside = 0;
    o->power = o->power_ref = 0.0;
    v3 s = ld3(s_in);
    if (!(s.z > 0.0)) return;                      /* no sun: nothing reaches the generator */
    or_view V;
    view_setup(P, s, n, centre, radius, &V);
    /* module terms: incidence, beam on the plane, depth bias */
    for (int64_t m = 0; m < P->n_mod; m++) {
        v3 nh = unit_normal(P, m);
        double cm = dot3(nh, s);
        beam[m] = cm > 0.0 ? dni * cm : 0.0;        /* back-lit: no beam */
        bias[m] = -1;                               /* -1: samples not tested */
        if (!(cm > 0.0) || !V.valid) continue;
        double nx = dot3(nh, V.e1), ny = dot3(nh, V.e2), nz = dot3(nh, V.d);
        double gxs = (fabs(nx / nz) * V.izd) / V.itx;
        double gys = (fabs(ny / nz) * V.izd) / V.ity;
        double b = ceil((0.5 + 1.0 / 512.0) * (gxs + gys)) + 2.0;
        if (!(b <= (double)OR_DMAX)) b = (double)OR_DMAX;
        bias[m] = (int32_t)b;
    }
    if (V.valid) {
        /* draw the scene, then (optionally) the modules themselves */
        for (int64_t t = 0; t < P->n_tri + (P->occluders ? 2 * P->n_mod : 0); t++) {
            v3 c[3];
            if (t < P->n_tri) {
                for (int q = 0; q < 3; q++) c[q] = ld3(P->xyz + 3 * (int64_t)P->tri[3 * t + q]);
            } else {
                v3 mc[4];
                int64_t mt = t - P->n_tri;
                module_corners(P, mt / 2, mc);
                if (mt % 2 == 0) { c[0] = mc[0]; c[1] = mc[1]; c[2] = mc[2]; }
                else { c[0] = mc[0]; c[1] = mc[2]; c[2] = mc[3]; }
            }
            double lt[3][3];
            for (int q = 0; q < 3; q++) {
                v3 l = to_light(&V, c[q]);
                lt[q][0] = l.x; lt[q][1] = l.y; lt[q][2] = l.z;
            }
            raster_light_triangle(lt, n, o->map, NULL);
        }
        /* depth check of every sub-cell sample of every front-lit module */
        for (int64_t m = 0; m < P->n_mod; m++) {
            if (bias[m] < 0) continue;
            v3 O = ld3(P->org + 3 * m), U = ld3(P->eu + 3 * m), W = ld3(P->ev + 3 * m);
            v3 p0 = to_light(&V, O);
            v3 du = mk(dot3(U, V.e1) * V.itx, dot3(U, V.e2) * V.ity, dot3(U, V.d) * V.izd);
            v3 dv = mk(dot3(W, V.e1) * V.itx, dot3(W, V.e2) * V.ity, dot3(W, V.d) * V.izd);
            for (int32_t cv = 0; cv < P->n_cv; cv++)
                for (int32_t cu = 0; cu < P->n_cu; cu++) {
                    int64_t cell = m * cpm + (int64_t)cv * P->n_cu + cu;
                    uint32_t cnt = 0;
                    for (int32_t b = 0; b < k; b++)
                        for (int32_t a = 0; a < k; a++) {
                            double fu = ((double)(k * cu + a) + 0.5) / (double)(k * P->n_cu);
                            double fv = ((double)(k * cv + b) + 0.5) / (double)(k * P->n_cv);
                            double x = (p0.x + fu * du.x) + fv * dv.x;
                            double y = (p0.y + fu * du.y) + fv * dv.y;
                            double z = (p0.z + fu * du.z) + fv * dv.z;
                            int64_t i = (int64_t)floor(x), j = (int64_t)floor(y);
                            int64_t zs = (int64_t)floor(z);
                            if (i < 0 || i >= n || j < 0 || j >= n) {
                                o->outside++;
                                if (i < 0) i = 0;
                                if (i >= n) i = n - 1;
                                if (j < 0) j = 0;
                                if (j >= n) j = n - 1;
                            }
                            int shaded = zs > (int64_t)o->map[j * (int64_t)n + i] + (int64_t)bias[m];
                            if (shaded) {
                                cnt++;
                                if (o->bits) {
                                    int32_t si = b * k + a;
                                    o->bits[cell * words + si / 32] |= 1u << (si % 32);
                                }
                            }
                        }
                    o->counts[cell] = cnt;
                }
        }
    }
    if (P->diode) {
        o->power = generator_power_diode(P, beam, o->counts, k, d_poa, sc->cap, sc->sub_len);
        o->power_ref = generator_power_diode(P, beam, NULL, k, d_poa, sc->cap, sc->sub_len);
    } else {
        o->power = generator_power(P, beam, o->counts, k, d_poa, sc->cap);
        o->power_ref = generator_power(P, beam, NULL, k, d_poa, sc->cap);
    }
}

/* ------------------------------------------------------------------------ */
/* trackers                                                                 */
/* ------------------------------------------------------------------------ */
/* Sec. 3.4 evaluates a plant of two-axis trackers; the paper states no
 * tracking law. Reading taken: ideal tracking with no angle limits and no
 * backtracking. A tracker turns the modules assigned to it about its pivot P.
 * At rest its frame is u0 = a x z, v0 = a, n0 = z, a being its horizontal
 * axis; a module given at rest keeps its coordinates in that frame, which for
 * a sun s (unit, above the horizon) becomes
 *   kind 1, one horizontal axis a:  v' = a, n' = unit(s - (s.a) a), u' = v' x n'
 *   kind 2, two axes:               n' = s, u' = unit(z x s), v' = n' x u'
 * (u' = u0 when the sun is at the zenith, n' = z if s is along a). */
typedef struct { int32_t kind; v3 p, a; } or_tracker;

static v3 unit3(v3 v) {
    double l = sqrt(dot3(v, v));
    return mk(v.x / l, v.y / l, v.z / l);
}

static void tracker_frame(const or_tracker* T, v3 s, v3* u, v3* v, v3* n) {
    const v3 z = mk(0.0, 0.0, 1.0);
    if (T->kind == 1) {
        double sa = dot3(s, T->a);
        v3 q = mk(s.x - sa * T->a.x, s.y - sa * T->a.y, s.z - sa * T->a.z);
        *v = T->a;
        *n = dot3(q, q) > 1e-30 ? unit3(q) : z;
        *u = cross3(*v, *n);
    } else {
        v3 h = cross3(z, s);
        *n = s;
        *u = dot3(h, h) > 1e-30 ? unit3(h) : cross3(T->a, z);
        *v = cross3(*n, *u);
    }
}

/* coordinates (c0, c1, c2) in the frame (u, v, n): (c0 u + c1 v) + c2 n */
static v3 in_frame(double c0, double c1, double c2, v3 u, v3 v, v3 n) {
    return mk((c0 * u.x + c1 * v.x) + c2 * n.x, (c0 * u.y + c1 * v.y) + c2 * n.y,
              (c0 * u.z + c1 * v.z) + c2 * n.z);
}

/* Module m of the rest pose (org, eu, ev) posed for sun s: untouched when it
 * belongs to no tracker (mod_trk[m] < 0). */
static void pose_module(const or_tracker* trk, const int32_t* mod_trk, const double* org, const double* eu,
                        const double* ev, int64_t m, v3 s, double* o_out, double* u_out, double* v_out) {
    v3 o = ld3(org + 3 * m), U = ld3(eu + 3 * m), W = ld3(ev + 3 * m);
    if (mod_trk[m] >= 0) {
        const or_tracker* T = trk + mod_trk[m];
        const v3 z = mk(0.0, 0.0, 1.0);
        v3 u0 = cross3(T->a, z), v0 = T->a, n0 = z, u, v, n;
        tracker_frame(T, s, &u, &v, &n);
        v3 r = sub3(o, T->p);
        o = add3(T->p, in_frame(dot3(r, u0), dot3(r, v0), dot3(r, n0), u, v, n));
        U = in_frame(dot3(U, u0), dot3(U, v0), dot3(U, n0), u, v, n);
        W = in_frame(dot3(W, u0), dot3(W, v0), dot3(W, n0), u, v, n);
    }
    o_out[0] = o.x; o_out[1] = o.y; o_out[2] = o.z;
    u_out[0] = U.x; u_out[1] = U.y; u_out[2] = U.z;
    v_out[0] = W.x; v_out[1] = W.y; v_out[2] = W.z;
}

/* Bounding sphere when modules move: the box of the scene vertices, the
 * corners of the modules that stay put, and for every tracker the cube
 * P +- r, r the distance from P of its farthest module corner at rest (a
 * rotation about P keeps every corner within it). */
static void tracked_sphere(const or_problem* P, const or_tracker* trk, int32_t n_trk, const int32_t* mod_trk,
                           v3* centre, double* radius) {
    v3 lo = mk(INFINITY, INFINITY, INFINITY), hi = mk(-INFINITY, -INFINITY, -INFINITY);
#define OR_GROW(q) do { v3 q_ = (q); \
        lo.x = q_.x < lo.x ? q_.x : lo.x; hi.x = q_.x > hi.x ? q_.x : hi.x; \
        lo.y = q_.y < lo.y ? q_.y : lo.y; hi.y = q_.y > hi.y ? q_.y : hi.y; \
        lo.z = q_.z < lo.z ? q_.z : lo.z; hi.z = q_.z > hi.z ? q_.z : hi.z; } while (0)
    for (int64_t i = 0; i < P->n_vert; i++) OR_GROW(ld3(P->xyz + 3 * i));
    for (int32_t t = 0; t < n_trk; t++) {
        double r = 0.0;
        for (int64_t m = 0; m < P->n_mod; m++) {
            if (mod_trk[m] != t) continue;
            v3 c[4];
            module_corners(P, m, c);
            for (int q = 0; q < 4; q++) {
                v3 d = sub3(c[q], trk[t].p);
                double l = sqrt(dot3(d, d));
                r = l > r ? l : r;
            }
        }
        if (r > 0.0) {
            OR_GROW(mk(trk[t].p.x - r, trk[t].p.y - r, trk[t].p.z - r));
            OR_GROW(mk(trk[t].p.x + r, trk[t].p.y + r, trk[t].p.z + r));
        }
    }
    for (int64_t m = 0; m < P->n_mod; m++) {
        if (mod_trk[m] >= 0) continue;
        v3 c[4];
        module_corners(P, m, c);
        for (int q = 0; q < 4; q++) OR_GROW(c[q]);
    }
#undef OR_GROW
    *centre = mk((lo.x + hi.x) * 0.5, (lo.y + hi.y) * 0.5, (lo.z + hi.z) * 0.5);
    v3 dg = sub3(hi, lo);
    *radius = 0.5 * sqrt(dot3(dg, dg));
}

static void read_trackers(const double* trk_in, int32_t n_trk, or_tracker* trk) {
    for (int32_t t = 0; t < n_trk; t++) {
        trk[t].kind = (int32_t)trk_in[7 * t];
        trk[t].p = ld3(trk_in + 7 * t + 1);
        trk[t].a = ld3(trk_in + 7 * t + 4);
    }
}

/* ------------------------------------------------------------------------ */
/* exported entry points (called through ctypes by the tests)               */
/* ------------------------------------------------------------------------ */
static void fill_problem(or_problem* P, const double* xyz, int64_t n_vert, const int32_t* tri,
                         int64_t n_tri, const double* org, const double* eu, const double* ev,
                         int64_t n_mod, int32_t n_cu, int32_t n_cv, const int32_t* cell_sub,
                         int32_t n_sub, const int32_t* mod_string, int32_t occluders) {
    P->xyz = xyz; P->n_vert = n_vert; P->tri = tri; P->n_tri = n_tri;
    P->org = org; P->eu = eu; P->ev = ev; P->n_mod = n_mod;
    P->n_cu = n_cu; P->n_cv = n_cv; P->cell_sub = cell_sub; P->n_sub = n_sub;
    P->mod_string = mod_string; P->occluders = occluders;
    P->diode = NULL;
    P->svf = NULL;
    int32_t ns = 0;
    for (int64_t m = 0; m < n_mod; m++)
        if (mod_string[m] + 1 > ns) ns = mod_string[m] + 1;
    P->n_string = ns;
}

/* Whole sweep. counts [n_sun][n_cells]; power, power_ref [n_sun]; energy[2] =
 * (sum P dt, sum P_ref dt) in sun order. depth_maps ([n_sun][n][n]) and bits
 * ([n_sun][n_cells][ceil(k*k/32)]) may be NULL. diode: single-diode cell
 * parameters (NULL: ideal strings); svf: [n_cells] sky view factors scaling
 * each cell's diffuse (NULL: 1). Returns the number of samples that fell
 * outside the map (0 when the window is right), or -1 on bad args. */
int64_t oracle_evaluate(const double* xyz, int64_t n_vert, const int32_t* tri, int64_t n_tri,
                        const double* org, const double* eu, const double* ev, int64_t n_mod,
                        int32_t n_cu, int32_t n_cv, const int32_t* cell_sub, int32_t n_sub,
                        const int32_t* mod_string, int32_t occluders,
                        const double* sun_xyz, const double* dni, const double* d_poa,
                        const double* dt_h, int64_t n_sun, int32_t n, int32_t k,
                        uint32_t* counts, double* power, double* power_ref, double* energy,
                        uint32_t* depth_maps, uint32_t* bits, int32_t threads, const double* diode,
                        const double* svf) {
    if (n < 16 || k < 1 || n_mod < 1) return -1;
    or_problem P;
    fill_problem(&P, xyz, n_vert, tri, n_tri, org, eu, ev, n_mod, n_cu, n_cv, cell_sub, n_sub,
                 mod_string, occluders);
    P.diode = diode;
    P.svf = svf;
    v3 centre;
    double radius;
    scene_sphere(&P, &centre, &radius);
    int64_t cells = n_mod * (int64_t)n_cu * n_cv;
    int32_t words = (k * k + 31) / 32;
    int64_t outside = 0;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#else
    (void)threads;
#endif
#pragma omp parallel reduction(+ : outside)
    {
        double* beam = (double*)malloc(sizeof(double) * (size_t)n_mod);
        int32_t* bias = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_mod);
        or_scratch sc;
        sc.cap = (double*)malloc(sizeof(double) * (size_t)cells);
        sc.sub_len = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_mod * n_sub));
        uint32_t* own_map = depth_maps ? NULL : (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n * n);
#pragma omp for schedule(dynamic, 1)
        for (int64_t t = 0; t < n_sun; t++) {
            or_sun_out o;
            o.counts = counts + t * cells;
            o.bits = bits ? bits + t * cells * words : NULL;
            o.map = depth_maps ? depth_maps + t * (int64_t)n * n : own_map;
            eval_sun(&P, centre, radius, sun_xyz + 3 * t, dni[t], d_poa[t], n, k, &o, beam, bias, &sc);
            power[t] = o.power;
            power_ref[t] = o.power_ref;
            outside += o.outside;
        }
        free(beam); free(bias); free(sc.cap); free(sc.sub_len); free(own_map);
    }
    double e = 0.0, er = 0.0;
    for (int64_t t = 0; t < n_sun; t++) {
        e += power[t] * dt_h[t];
        er += power_ref[t] * dt_h[t];
    }
    energy[0] = e;
    energy[1] = er;
    return outside;
}

/* ------------------------------------------------------------------------ */
/* diffuse shading: sky view factors                                        */
/* ------------------------------------------------------------------------ */
/* The paper's evaluation removes only the beam from shaded areas and notes
 * that obstacles also hide part of the diffuse sky (Sec. 4). Reading taken:
 * an isotropic sky seen through a fixed set of directions s_j above the
 * horizon, each standing for an equal share of it. A sample sees direction j
 * when the depth test from s_j finds it lit. A cell's sky view factor is
 *   svf = sum_j w_j (1 - shaded_j / k^2) / sum_j w_j,  w_j = max(0, n . s_j),
 * n the module's front normal, summed in direction order; 1 when no direction
 * lies in front of the module. The diffuse a cell receives is then
 * d_poa * svf. Every direction is evaluated as a sun of unit beam: the same
 * view, depth picture and test. dirs: [n_dir][3] unit vectors with z > 0.
 * svf_out: [n_cells]. Returns the samples that fell outside a map, or -1. */
int64_t oracle_sky_view(const double* xyz, int64_t n_vert, const int32_t* tri, int64_t n_tri,
                        const double* org, const double* eu, const double* ev, int64_t n_mod,
                        int32_t n_cu, int32_t n_cv, const int32_t* cell_sub, int32_t n_sub,
                        const int32_t* mod_string, int32_t occluders, const double* dirs, int64_t n_dir,
                        int32_t n, int32_t k, double* svf_out, int32_t threads) {
    if (n < 16 || k < 1 || n_mod < 1 || n_dir < 1) return -1;
    for (int64_t j = 0; j < n_dir; j++)
        if (!(dirs[3 * j + 2] > 0.0)) return -1;
    int64_t cells = n_mod * (int64_t)n_cu * n_cv;
    uint32_t* counts = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(cells * n_dir));
    double* in = (double*)malloc(sizeof(double) * (size_t)n_dir * 3);   /* beam 1, no diffuse, no weight */
    for (int64_t j = 0; j < n_dir; j++) { in[j] = 1.0; in[n_dir + j] = 0.0; in[2 * n_dir + j] = 0.0; }
    double* pw = (double*)malloc(sizeof(double) * (size_t)n_dir * 2);
    double en[2];
    int64_t out = oracle_evaluate(xyz, n_vert, tri, n_tri, org, eu, ev, n_mod, n_cu, n_cv, cell_sub, n_sub,
                                  mod_string, occluders, dirs, in, in + n_dir, in + 2 * n_dir, n_dir, n, k,
                                  counts, pw, pw + n_dir, en, NULL, NULL, threads, NULL, NULL);
    if (out >= 0) {
        or_problem P;
        fill_problem(&P, xyz, n_vert, tri, n_tri, org, eu, ev, n_mod, n_cu, n_cv, cell_sub, n_sub,
                     mod_string, occluders);
        int64_t cpm = (int64_t)n_cu * n_cv;
        for (int64_t m = 0; m < n_mod; m++) {
            v3 nh = unit_normal(&P, m);
            for (int64_t c = 0; c < cpm; c++) {
                double num = 0.0, den = 0.0;
                for (int64_t j = 0; j < n_dir; j++) {
                    double w = dot3(nh, ld3(dirs + 3 * j));
                    if (!(w > 0.0)) continue;
                    double f = (double)counts[j * cells + m * cpm + c] / (double)(k * k);
                    num += w * (1.0 - f);
                    den += w;
                }
                svf_out[m * cpm + c] = den > 0.0 ? num / den : 1.0;
            }
        }
    }
    free(counts); free(in); free(pw);
    return out;
}

/* View and module terms of one sun, for the tests' brute-force comparison.
 * view_out[17] = e1(3) e2(3) d(3) ox oy itx ity znear izd valid n;
 * beam_out, bias_out [n_mod] (bias -1: back-lit). */
void oracle_view(const double* xyz, int64_t n_vert, const double* org, const double* eu,
                 const double* ev, int64_t n_mod, const double* sun, double dni, int32_t n,
                 double* view_out, double* beam_out, int32_t* bias_out) {
    or_problem P;
    memset(&P, 0, sizeof(P));
    P.xyz = xyz; P.n_vert = n_vert; P.org = org; P.eu = eu; P.ev = ev; P.n_mod = n_mod;
    v3 centre;
    double radius;
    scene_sphere(&P, &centre, &radius);
    or_view V;
    view_setup(&P, ld3(sun), n, centre, radius, &V);
    double* w = view_out;
    w[0] = V.e1.x; w[1] = V.e1.y; w[2] = V.e1.z;
    w[3] = V.e2.x; w[4] = V.e2.y; w[5] = V.e2.z;
    w[6] = V.d.x; w[7] = V.d.y; w[8] = V.d.z;
    w[9] = V.ox; w[10] = V.oy; w[11] = V.itx; w[12] = V.ity; w[13] = V.znear; w[14] = V.izd;
    w[15] = (double)V.valid; w[16] = (double)n;
    v3 s = ld3(sun);
    for (int64_t m = 0; m < n_mod; m++) {
        v3 nh = unit_normal(&P, m);
        double cm = dot3(nh, s);
        beam_out[m] = cm > 0.0 ? dni * cm : 0.0;
        bias_out[m] = -1;
        if (!(cm > 0.0) || !V.valid) continue;
        double nx = dot3(nh, V.e1), ny = dot3(nh, V.e2), nz = dot3(nh, V.d);
        double b = ceil((0.5 + 1.0 / 512.0) * ((fabs(nx / nz) * V.izd) / V.itx +
                                               (fabs(ny / nz) * V.izd) / V.ity)) + 2.0;
        if (!(b <= (double)OR_DMAX)) b = (double)OR_DMAX;
        bias_out[m] = (int32_t)b;
    }
}

/* Raster triangles given directly in light space ([n_tri][3][3]: x, y in
 * texels, z in depth units) into map (initialised to 2^24-1 here) and count
 * how many triangles cover each pixel centre (cover may be NULL). */
void oracle_raster(const double* tris, int64_t n_tri, int32_t n, uint32_t* map, uint32_t* cover) {
    for (int64_t p = 0; p < (int64_t)n * n; p++) {
        map[p] = OR_DMAX;
        if (cover) cover[p] = 0;
    }
    for (int64_t t = 0; t < n_tri; t++) {
        double lt[3][3];
        for (int q = 0; q < 3; q++)
            for (int k = 0; k < 3; k++) lt[q][k] = tris[9 * t + 3 * q + k];
        raster_light_triangle(lt, n, map, cover);
    }
}

/* Ideal bypass string power of given substring capacities (for pins). */
double oracle_string_power(const double* caps, int64_t n) {
    double* c = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    memcpy(c, caps, sizeof(double) * (size_t)n);
    double p = string_power(c, n);
    free(c);
    return p;
}

/* Single-diode model pieces (for pins): the voltage of one cell, and the
 * maximum power of one string whose cells' irradiances g are given substring
 * after substring (sub_len cells each, n_q substrings). d as above. */
double oracle_cell_voltage(const double* d, double G, double I) { return cell_voltage(d, G, I); }

double oracle_string_voltage(const double* d, const double* g, const int32_t* sub_len, int64_t n_q, double I) {
    return string_voltage(d, g, sub_len, n_q, I);
}

double oracle_string_mpp(const double* d, const double* g, const int32_t* sub_len, int64_t n_q) {
    return string_mpp(d, g, sub_len, n_q);
}

/* Rest-pose modules (org, eu, ev) posed for one sun: trk [n_trk][7] = kind,
 * pivot xyz, axis xyz; mod_trk [n_mod] the tracker of each module (-1 none). */
void oracle_pose(const double* trk_in, int32_t n_trk, const int32_t* mod_trk, const double* org,
                 const double* eu, const double* ev, int64_t n_mod, const double* sun,
                 double* org_out, double* eu_out, double* ev_out) {
    or_tracker* trk = (or_tracker*)malloc(sizeof(or_tracker) * (size_t)(n_trk > 0 ? n_trk : 1));
    read_trackers(trk_in, n_trk, trk);
    v3 s = ld3(sun);
    for (int64_t m = 0; m < n_mod; m++)
        pose_module(trk, mod_trk, org, eu, ev, m, s, org_out + 3 * m, eu_out + 3 * m, ev_out + 3 * m);
    free(trk);
}

/* oracle_evaluate for a generator whose modules follow the sun: every sun is
 * evaluated with the modules posed for it (bounding sphere as above). */
int64_t oracle_evaluate_tracked(const double* xyz, int64_t n_vert, const int32_t* tri, int64_t n_tri,
                                const double* org, const double* eu, const double* ev, int64_t n_mod,
                                int32_t n_cu, int32_t n_cv, const int32_t* cell_sub, int32_t n_sub,
                                const int32_t* mod_string, int32_t occluders,
                                const double* trk_in, int32_t n_trk, const int32_t* mod_trk,
                                const double* sun_xyz, const double* dni, const double* d_poa,
                                const double* dt_h, int64_t n_sun, int32_t n, int32_t k,
                                uint32_t* counts, double* power, double* power_ref, double* energy,
                                uint32_t* depth_maps, uint32_t* bits, int32_t threads, const double* diode,
                        const double* svf) {
    if (n < 16 || k < 1 || n_mod < 1 || n_trk < 0) return -1;
    for (int64_t m = 0; m < n_mod; m++)
        if (mod_trk[m] >= n_trk) return -1;
    or_problem P;
    fill_problem(&P, xyz, n_vert, tri, n_tri, org, eu, ev, n_mod, n_cu, n_cv, cell_sub, n_sub,
                 mod_string, occluders);
    P.diode = diode;
    P.svf = svf;
    or_tracker* trk = (or_tracker*)malloc(sizeof(or_tracker) * (size_t)(n_trk > 0 ? n_trk : 1));
    read_trackers(trk_in, n_trk, trk);
    v3 centre;
    double radius;
    tracked_sphere(&P, trk, n_trk, mod_trk, &centre, &radius);
    int64_t cells = n_mod * (int64_t)n_cu * n_cv;
    int32_t words = (k * k + 31) / 32;
    int64_t outside = 0;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
#else
    (void)threads;
#endif
#pragma omp parallel reduction(+ : outside)
    {
        double* beam = (double*)malloc(sizeof(double) * (size_t)n_mod);
        int32_t* bias = (int32_t*)malloc(sizeof(int32_t) * (size_t)n_mod);
        or_scratch sc;
        sc.cap = (double*)malloc(sizeof(double) * (size_t)cells);
        sc.sub_len = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n_mod * n_sub));
        double* pose = (double*)malloc(sizeof(double) * (size_t)(9 * n_mod));
        uint32_t* own_map = depth_maps ? NULL : (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n * n);
#pragma omp for schedule(dynamic, 1)
        for (int64_t t = 0; t < n_sun; t++) {
            v3 s = ld3(sun_xyz + 3 * t);
            or_problem Ps = P;
            if (s.z > 0.0) {
                for (int64_t m = 0; m < n_mod; m++)
                    pose_module(trk, mod_trk, org, eu, ev, m, s, pose + 3 * m, pose + 3 * (n_mod + m),
                                pose + 3 * (2 * n_mod + m));
                Ps.org = pose;
                Ps.eu = pose + 3 * n_mod;
                Ps.ev = pose + 6 * n_mod;
            }
            or_sun_out o;
            o.counts = counts + t * cells;
            o.bits = bits ? bits + t * cells * words : NULL;
            o.map = depth_maps ? depth_maps + t * (int64_t)n * n : own_map;
            eval_sun(&Ps, centre, radius, sun_xyz + 3 * t, dni[t], d_poa[t], n, k, &o, beam, bias, &sc);
            power[t] = o.power;
            power_ref[t] = o.power_ref;
            outside += o.outside;
        }
        free(beam); free(bias); free(sc.cap); free(sc.sub_len); free(pose); free(own_map);
    }
    free(trk);
    double e = 0.0, er = 0.0;
    for (int64_t t = 0; t < n_sun; t++) {
        e += power[t] * dt_h[t];
        er += power_ref[t] * dt_h[t];
    }
    energy[0] = e;
    energy[1] = er;
    return outside;
}
