"""Pins of the CPU oracle against what geometry and the paper fix (CPU only).

Each test checks the oracle against something other than itself: exact ray
casting, closed-form shadow lengths, exact rational arithmetic, invariants of
the method (nearest depth wins, shading only removes the beam), or brute force
over a tiny input.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_1410_5780_amd import workloads as W
from tests import _geom as G

DMAX = (1 << 24) - 1


def run(oracle_lib, w, **kw):
    r = oracle_lib.evaluate(w.scene, w.gen, w.sweep, w.map_n, w.k, **kw)
    assert r.outside == 0, "a sample fell outside the window"
    return r


# --------------------------------------------------------------------------
# C1: one module, one pole, day 355 (closed forms)
# --------------------------------------------------------------------------
def test_c1_matches_exact_ray_casting(oracle_lib):
    """Every sample of every up-hour agrees with exact ray/box occlusion (no band needed)."""
    w = W.c1_tiny()
    r = run(oracle_lib, w, export_bits=True)
    pts = G.sample_points(w.gen, w.k).reshape(-1, 3)            # (cv, cu, b, a) order
    box = w.scene.xyz[w.scene.tri]
    for h in range(24):
        s = w.sweep.sun_xyz[h]
        got = G.unpack_bits(r.bits[h], w.k)                      # [cell, b*k+a]
        if s[2] <= 0:
            assert not got.any() and r.power[h] == 0 and r.power_ref[h] == 0
            continue
        exact = np.isfinite(G.ray_hits(pts, s, box)).any(axis=1).reshape(60, w.k * w.k)
        assert np.array_equal(got, exact), f"hour {h}"
    assert list(r.counts.sum(axis=1)) == [0] * 12 + [3200] + [0] * 11
    noon = r.counts[12].reshape(10, 6)
    assert np.all(noon[:, 2:4] == 160) and noon[:, [0, 1, 4, 5]].sum() == 0
    assert np.all(noon[:, 2:4] / 256.0 == 0.625)


@pytest.mark.parametrize("d_poa,want", [(0.0, 0.04822617), (100.0, 0.04670964)])
def test_c1_loss_closed_form(oracle_lib, d_poa, want):
    """Only noon is shaded: substring 1 drops to 0.375 of the beam, the string keeps 2 of 3
    substrings, so the day loses (B_noon + D) / sum_t 3 (B_t + D)."""
    w = W.c1_tiny(d_poa=d_poa)
    r = run(oracle_lib, w)
    n = np.array([0.0, -math.sin(math.radians(30)), math.cos(math.radians(30))])
    cos = w.sweep.sun_xyz @ n
    up = (w.sweep.sun_xyz[:, 2] > 0) & (cos > 0)
    beam = np.where(up, 1000.0 * cos, 0.0)
    ref = np.where(w.sweep.sun_xyz[:, 2] > 0, 3 * (beam + d_poa), 0.0)
    loss = (beam[12] + d_poa) / ref.sum()
    assert r.loss == pytest.approx(loss, rel=1e-12)
    assert r.loss == pytest.approx(want, abs=5e-9)
    assert np.allclose(r.power_ref, ref, rtol=1e-14)
    p = ref.copy()
    p[12] = 2 * (beam[12] + d_poa)
    assert np.allclose(r.power, p, rtol=1e-14)
    assert r.energy[1] == pytest.approx(ref.sum(), rel=1e-14)


# --------------------------------------------------------------------------
# electrical model
# --------------------------------------------------------------------------
def test_string_power_is_best_operating_current(oracle_lib):
    """Ideal bypass string: P(I) = I * #{substrings able to carry I}; the oracle returns its max."""
    rng = np.random.default_rng(0)
    for trial in range(200):
        n = int(rng.integers(1, 25))
        caps = rng.choice([rng.uniform(0, 1000, n), np.round(rng.uniform(0, 5, n)) * 100.0])
        grid = np.concatenate([caps, np.linspace(0, caps.max(), 2001)])
        best = max(float(I) * int((caps >= I).sum()) for I in grid)
        assert oracle_lib.string_power(caps) == pytest.approx(best, rel=1e-15, abs=0)
    assert oracle_lib.string_power(np.full(7, 3.5)) == 7 * 3.5
    assert oracle_lib.string_power(np.array([5.0, 0.0, 5.0])) == 10.0
    assert oracle_lib.string_power(np.array([10.0, 1.0, 1.0])) == 10.0


# --------------------------------------------------------------------------
# rasterization: fill rule and depth
# --------------------------------------------------------------------------
def _grid_mesh(rng, x0, y0, nx, ny, step, jitter):
    xs = x0 + step * np.arange(nx + 1)
    ys = y0 + step * np.arange(ny + 1)
    X, Y = np.meshgrid(xs, ys, indexing="ij")
    X = X.copy(); Y = Y.copy()
    inner = (slice(1, nx), slice(1, ny))
    X[inner] += rng.uniform(-jitter, jitter, X[inner].shape)
    Y[inner] += rng.uniform(-jitter, jitter, Y[inner].shape)
    Z = rng.uniform(100, 1000, X.shape)
    P = np.stack([X, Y, Z], -1)
    tris = []
    for i in range(nx):
        for j in range(ny):
            a, b, c, d = P[i, j], P[i + 1, j], P[i + 1, j + 1], P[i, j + 1]
            if rng.random() < 0.5:
                tris += [(a, b, c), (a, c, d)]
            else:
                tris += [(a, b, d), (b, c, d)]
    tris = np.array(tris)
    flip = rng.random(len(tris)) < 0.5                 # random winding
    tris[flip] = tris[flip][:, ::-1]
    return tris


@pytest.mark.parametrize("seed,x0,y0,step,jitter", [
    (0, 10.5, 7.5, 4.0, 0.0),          # every vertex on a pixel centre: shared edges through centres
    (1, 10.5, 7.5, 3.0, 0.6),          # jittered interior (below step/4: no fold)
    (2, 3.25, 5.0, 2.5, 0.55),
    (3, 0.5, 0.5, 1.0, 0.0),           # unit squares on centres: every centre is a shared vertex
])
def test_fill_rule_covers_each_centre_once(oracle_lib, seed, x0, y0, step, jitter):
    rng = np.random.default_rng(seed)
    nx, ny, n = 12, 10, 64
    tris = _grid_mesh(rng, x0, y0, nx, ny, step, jitter)
    _, cover = oracle_lib.raster(tris, n)
    x1, y1 = x0 + nx * step, y0 + ny * step
    c = np.arange(n) + 0.5
    cx, cy = c[None, :], c[:, None]                    # cover[j, i]
    inside = (cx > x0) & (cx < x1) & (cy > y0) & (cy < y1)
    # boundary of the union: left and top edges are in, right and bottom out (y up)
    on_left = (cx == x0) & (cy > y0) & (cy <= y1)
    on_top = (cy == y1) & (cx >= x0) & (cx < x1)
    want = (inside | on_left | on_top).astype(np.uint32)
    assert cover.max() <= 1
    assert np.array_equal(cover, want)


def test_fan_around_a_pixel_centre(oracle_lib):
    """Eight triangles sharing a vertex exactly at a pixel centre: it is covered exactly once."""
    c = np.array([20.5, 20.5, 50.0])
    ring = [np.array([20.5 + 9 * math.cos(a), 20.5 + 9 * math.sin(a), 60.0])
            for a in np.linspace(0, 2 * np.pi, 9)[:-1]]
    tris = np.array([(c, ring[q], ring[(q + 1) % 8]) for q in range(8)])
    _, cover = oracle_lib.raster(tris, 48)
    assert cover[20, 20] == 1
    assert cover.max() == 1


def _exact_depth_floor(tri, i, j):
    X = [math.floor(Fraction(v[0]) * 256 + Fraction(1, 2)) for v in tri]
    Y = [math.floor(Fraction(v[1]) * 256 + Fraction(1, 2)) for v in tri]
    Z = [Fraction(v[2]) for v in tri]
    i, j = int(i), int(j)
    px, py = Fraction(2 * i + 1, 2), Fraction(2 * j + 1, 2)
    x = [Fraction(a, 256) for a in X]
    y = [Fraction(a, 256) for a in Y]
    den = (x[1] - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (y[1] - y[0])
    l1 = ((px - x[0]) * (y[2] - y[0]) - (x[2] - x[0]) * (py - y[0])) / den
    l2 = ((x[1] - x[0]) * (py - y[0]) - (px - x[0]) * (y[1] - y[0])) / den
    z = Z[0] + l1 * (Z[1] - Z[0]) + l2 * (Z[2] - Z[0])
    return math.floor(z)


def test_depth_within_one_unit_of_exact_plane(oracle_lib):
    rng = np.random.default_rng(5)
    n = 40
    checked = 0
    for t in range(60):
        tri = np.concatenate([rng.uniform(-5, n + 5, (3, 2)), rng.uniform(0, 3e6, (3, 1))], 1)
        m, cover = oracle_lib.raster(tri[None], n)
        js, is_ = np.nonzero(cover)
        for j, i in list(zip(js, is_))[:40]:
            e = min(max(_exact_depth_floor(tri, i, j), 0), DMAX)
            assert abs(int(m[j, i]) - e) <= 1, (t, i, j, int(m[j, i]), e)
            checked += 1
    assert checked > 500


def test_nearest_depth_wins_and_order_does_not_matter(oracle_lib):
    rng = np.random.default_rng(9)
    n = 48
    tris = np.concatenate([rng.uniform(-3, n + 3, (80, 3, 2)), rng.uniform(0, DMAX * 1.2, (80, 3, 1))], 2)
    full, _ = oracle_lib.raster(tris, n)
    perm, _ = oracle_lib.raster(tris[rng.permutation(80)], n)
    assert np.array_equal(full, perm)
    singles = np.stack([oracle_lib.raster(t[None], n, with_cover=False)[0] for t in tris])
    assert np.array_equal(full, singles.min(axis=0))


def test_guard_band_clip_keeps_coverage_and_plane(oracle_lib):
    """A triangle reaching 2^25 texels out is clipped to the guard square; inside the map it
    still covers every centre once and keeps its plane within one depth unit."""
    n = 32
    big = 2.0 ** 25
    z = lambda x, y: 5000.0 + 0.25 * x - 0.125 * y
    v = np.array([[-big, -big], [big, -big * 0.5], [0.3 * big, big]])
    tri = np.array([[p[0], p[1], z(p[0], p[1])] for p in v])
    m, cover = oracle_lib.raster(tri[None], n)
    assert np.all(cover == 1)
    ii, jj = np.meshgrid(np.arange(n) + 0.5, np.arange(n) + 0.5)
    assert np.max(np.abs(m.astype(np.int64) - np.floor(z(ii, jj)))) <= 1


# --------------------------------------------------------------------------
# invariants of the shading step
# --------------------------------------------------------------------------
def test_generator_alone_is_never_shaded(oracle_lib):
    """Coplanar modules with nothing else around: the depth bias keeps every sample lit."""
    yr = W.year_sweep().subset(np.arange(0, 4379, 37))
    c1 = W.c1_tiny()
    alone = W.Workload("alone", W.Scene(np.zeros((0, 3)), np.zeros((0, 3), np.int32)), c1.gen, yr, 512, 4)
    r = run(oracle_lib, alone)
    assert r.counts.sum() == 0 and np.array_equal(r.power, r.power_ref)
    flat = W.c3_rooftop(sweep=yr, n_buildings=0, n_trees=0, map_n=1024, k=2)
    flat.gen.origin[:, 2] += 0.0
    flat = W.Workload("flat", W.Scene(np.zeros((0, 3)), np.zeros((0, 3), np.int32)),
                      flat.gen, yr, 1024, 2)
    r = run(oracle_lib, flat)
    assert r.counts.sum() == 0


def test_below_horizon_contributes_nothing(oracle_lib):
    w = W.c1_tiny(d_poa=100.0)
    w.sweep = W.make_sweep(40.4, [355, 172], [0.0, 3.0, 21.0, 23.0], d_poa=100.0)
    r = run(oracle_lib, w, export_maps=True)
    assert r.counts.sum() == 0 and r.power.sum() == 0 and r.power_ref.sum() == 0
    assert np.all(r.maps == DMAX) and r.energy[0] == 0 and r.energy[1] == 0


def test_adding_occluders_only_darkens(oracle_lib):
    base = W.random_tiny(11, n_boxes=4, n_loose=10, n_sun=5, map_n=160, k=4)
    more = W.random_tiny(11, n_boxes=4, n_loose=10, n_sun=5, map_n=160, k=4)
    rng = np.random.default_rng(3)
    lo, hi = base.scene.xyz.min(0), base.scene.xyz.max(0)
    extra = rng.uniform(lo, hi, (15, 3, 3)).reshape(-1, 3)
    more.scene = W.Scene(np.concatenate([base.scene.xyz, extra]),
                         np.concatenate([base.scene.tri, base.scene.n_vert + np.arange(45).reshape(15, 3)]).astype(np.int32))
    a = run(oracle_lib, base, export_maps=True)
    b = run(oracle_lib, more, export_maps=True)
    assert np.all(b.maps <= a.maps) and np.all(b.counts >= a.counts)
    assert np.all(b.power <= a.power + 1e-9) and np.array_equal(a.power_ref, b.power_ref)


def test_triangle_order_does_not_change_results(oracle_lib):
    w = W.random_tiny(12, n_boxes=8, n_loose=25, n_sun=4, map_n=150, k=3)
    a = run(oracle_lib, w, export_maps=True, export_bits=True)
    rng = np.random.default_rng(1)
    w.scene = W.Scene(w.scene.xyz, np.ascontiguousarray(w.scene.tri[rng.permutation(w.scene.n_tri)]))
    b = run(oracle_lib, w, export_maps=True, export_bits=True)
    assert np.array_equal(a.maps, b.maps) and np.array_equal(a.bits, b.bits)
    assert np.array_equal(a.power, b.power)


# --------------------------------------------------------------------------
# closed-form shadow lengths
# --------------------------------------------------------------------------
@pytest.mark.parametrize("day", [355, 172])
def test_pole_shadow_length_on_flat_receiver(oracle_lib, day):
    """A 4 m pole on a horizontal receiver: at noon its shadow reaches H cot(elevation)
    beyond the pole's north face."""
    H = 4.0
    nx, ny = 4, 24
    O = np.array([[-2.0 + 1.0 * i, 0.0 + 0.5 * j, 0.0] for j in range(ny) for i in range(nx)])
    gen = W.Generator(O, np.tile([1.0, 0, 0], (nx * ny, 1)), np.tile([0, 0.5, 0.0], (nx * ny, 1)),
                      2, 2, np.array([0, 0, 1, 1], np.int32), 2, np.zeros(nx * ny, np.int32),
                      add_as_occluders=False)
    v, t = W.boxes(0.0, -0.2, 0.2, 0.2, -0.5, H, 0.0)
    sw = W.make_sweep(40.4, [day], [12.0])
    k = 8
    w = W.Workload("pole", W.Scene(v[0], t.astype(np.int32)), gen, sw, 2048, k)
    r = run(oracle_lib, w, export_bits=True)
    bits = G.unpack_bits(r.bits[0], k).reshape(-1)
    pts = G.sample_points(gen, k).reshape(-1, 3)
    shaded = pts[bits]
    elev = math.asin(sw.sun_xyz[0, 2])
    tip = -0.1 + H / math.tan(elev)
    ny_px = 12.0 / (2048 - 2)
    tol = ny_px + 0.5 / k + 1e-9
    centre = np.abs(shaded[:, 0]) < 0.05
    assert shaded[centre, 1].max() == pytest.approx(tip, abs=tol)
    assert np.all(np.abs(shaded[:, 0]) < 0.1 + 1.0 / k)


def test_inter_row_shading_closed_form(oracle_lib):
    """Parallel rows: the row in front shades l* = L - D sin(a) / sin(a + b) of the slant."""
    sw = W.make_sweep(40.4, [355], np.arange(8.0, 16.0))
    w = W.c2_row_plant(n_pylons=0, sweep=sw, map_n=2048, k=8, gap=0.0)   # continuous rows
    r = run(oracle_lib, w, export_bits=True)
    D, L, beta = 3.9, 1.56, math.radians(30)
    for t in range(sw.n):
        s = sw.sun_xyz[t]
        alpha = math.atan2(s[2], -s[1])
        lstar = max(0.0, L - D * math.sin(alpha) / math.sin(alpha + beta))
        want_rows = sum(1 for b in range(80) if (b + 0.5) / 80 * L < lstar)
        bits = G.unpack_bits(r.bits[t], 8).reshape(400, 10, 6, 8, 8)   # module, cv, cu, b, a
        for row in range(1, 20):
            for col in range(3, 10):
                m = row * 20 + col
                per_col = bits[m].transpose(1, 3, 0, 2).reshape(48, 80).sum(axis=1)
                assert np.all(np.abs(per_col - want_rows) <= 1), (t, row, col, want_rows, per_col)
        if 9 <= sw.hour[t] <= 15:
            assert r.counts[t].sum() == 0
    assert want_rows == 0
    first = G.unpack_bits(r.bits[0], 8).reshape(400, 10, 6, 8, 8)
    assert first[:20].sum() == 0                        # the front row is never shaded by rows


# --------------------------------------------------------------------------
# brute force on tiny random scenes, disagreements confined to the band
# --------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [21, 22, 23, 24])
def test_agrees_with_ray_casting_outside_band(oracle_lib, seed):
    w = W.random_tiny(seed, n_boxes=8, n_loose=30, n_mod_side=2, map_n=220, k=4, n_sun=6)
    r = run(oracle_lib, w, export_bits=True)
    tris, owner = G.all_triangles(w)
    pts = G.sample_points(w.gen, w.k).reshape(w.gen.n_mod, -1, 3)
    tot = dis = 0
    for t in range(w.sweep.n):
        s = w.sweep.sun_xyz[t]
        vw = oracle_lib.view(w.scene, w.gen, s, w.map_n)
        if not vw["valid"]:
            continue
        e1, e2, d = vw["e1"], vw["e2"], vw["d"]
        tx, ty = 1.0 / vw["itx"], 1.0 / vw["ity"]
        delta = 0.5 * math.hypot(tx, ty) + 2.0 ** -8 * max(tx, ty) + 1e-9
        bits = G.unpack_bits(r.bits[t], w.k).reshape(w.gen.n_mod, -1)
        for m in range(w.gen.n_mod):
            nrm = np.cross(w.gen.edge_u[m], w.gen.edge_v[m])
            nrm /= np.linalg.norm(nrm)
            if nrm @ s < 0.1:
                continue
            others = owner != m
            P = pts[m]
            hit = G.ray_hits(P, s, tris[others])
            exact = np.isfinite(hit).any(axis=1)
            got = bits[m]
            tot += got.size
            bad = np.nonzero(got != exact)[0]
            dis += bad.size
            if bad.size == 0:
                continue
            T = tris[others]
            tz = T @ d                                   # [m,3] depth along the view
            pu, pv, pz = P[bad] @ e1, P[bad] @ e2, P[bad] @ d
            Tu, Tv = T @ e1, T @ e2
            near_edge = np.zeros(bad.size, bool)
            for a_, b_ in ((0, 1), (1, 2), (2, 0)):
                dist = G.seg_dist(np.stack([pu, pv], 1), np.stack([Tu[:, a_], Tv[:, a_]], 1),
                                  np.stack([Tu[:, b_], Tv[:, b_]], 1))
                front = tz.min(axis=1)[None, :] < pz[:, None]
                near_edge |= ((dist <= delta) & front).any(axis=1)
            # depth band: the occluder met on the ray is within the bias plus its own slope
            tn = np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0])
            with np.errstate(divide="ignore", invalid="ignore"):
                slope = (np.abs((tn @ e1) / (tn @ d)) * vw["izd"] / vw["itx"]
                         + np.abs((tn @ e2) / (tn @ d)) * vw["izd"] / vw["ity"])
            slope = np.nan_to_num(slope, nan=np.inf, posinf=np.inf)
            gap = hit[bad] * vw["izd"]
            near_depth = (gap <= vw["bias"][m] + 2 + slope[None, :] * (0.5 * math.sqrt(2) + 2 ** -8)).any(axis=1)
            out = ~(near_edge | near_depth)
            assert not out.any(), f"sun {t} module {m}: {out.sum()} disagreements outside the band"
    assert tot > 5000
    assert dis / tot < 0.02


def test_back_lit_module_is_not_tested(oracle_lib):
    """A module whose back faces the sun receives no beam and has no shaded samples, even with
    an occluder between it and the sun (summer dawn: the sun is north of east). A second,
    north-facing module keeps the view open."""
    w = W.c1_tiny(d_poa=40.0)
    b = math.radians(30.0)
    g = w.gen
    g.origin = np.array([g.origin[0], [-7.0 + W.MOD_W / 2, W.MOD_L * math.cos(b), 0.0]])
    g.edge_u = np.array([g.edge_u[0], [-W.MOD_W, 0.0, 0.0]])
    g.edge_v = np.array([g.edge_v[0], [0.0, -W.MOD_L * math.cos(b), W.MOD_L * math.sin(b)]])
    g.module_string = np.array([0, 1], np.int32)
    v, t = W.boxes([4.0, -4.0], [2.5, 2.5], 1.0, 6.0, 0.0, 3.0, 0.0)   # walls east and west
    w.scene = W.Scene(v.reshape(-1, 3), np.concatenate([t, t + 8]).astype(np.int32))
    w.sweep = W.make_sweep(40.4, [172], [5.0, 19.0], d_poa=40.0)
    n = np.cross(w.gen.edge_u[0], w.gen.edge_v[0])
    n2 = np.cross(w.gen.edge_u[1], w.gen.edge_v[1])
    assert np.all(w.sweep.sun_xyz @ n < 0) and np.all(w.sweep.sun_xyz @ n2 > 0)
    assert np.all(w.sweep.sun_xyz[:, 2] > 0)
    pts = G.sample_points(w.gen, w.k)[0].reshape(-1, 3)
    for s in w.sweep.sun_xyz:                      # the walls do stand between sun and module 0
        assert np.isfinite(G.ray_hits(pts, s, w.scene.xyz[w.scene.tri])).any(axis=1).mean() > 0.5
    r = run(oracle_lib, w)
    assert r.counts[:, :60].sum() == 0
    # string 0 (the back-lit module) carries diffuse only: 3 substrings at 40 W/m^2
    r0 = oracle_lib.string_power(np.full(3, 40.0))
    assert np.all(r.power_ref - r.power >= 0) and r0 == 120.0
