"""Pins of the oracle on scenes with many generators (CPU only).

Sec. 3.3 evaluates each of many generators in one shared scene, with its own
orientation and surroundings. Every generator's modules are scene triangles,
so each is shaded by the others. Checked here: the shadows agree with exact ray
casting except within a texel of an occluder's outline; a generator's own
modules given as scene triangles act exactly as when the generator adds them
itself; and the stadium's shapes (sizes, non-overlap, orientation).
"""
import dataclasses
import math

import numpy as np

from paper_1410_5780_amd import workloads as W
from tests import _geom as G


def _unit(a):
    return a / np.linalg.norm(a, axis=-1, keepdims=True)


def test_stadium_shapes():
    sw = W.make_sweep(W.LAT_DEG, [172], [12.0])
    ws = W.c7_stadium(sweep=sw)
    assert len(ws) == 88
    sc = ws[0].scene
    assert all(w.scene is sc for w in ws), "one scene shared by every generator"
    assert all(w.gen.n_mod == 56 and w.gen.n_cells == 3360 and not w.gen.add_as_occluders for w in ws)
    # every generator's modules are in the scene, two triangles each, in generator order
    t = sc.xyz[sc.tri]
    for i in (0, 41, 87):
        g = ws[i].gen
        a = t[2 * 56 * i: 2 * 56 * i + 56]
        np.testing.assert_array_equal(a[:, 0], g.origin)
        np.testing.assert_array_equal(a[:, 2], (g.origin + g.edge_u) + g.edge_v)
    # planes face up, tilted 12 degrees toward the ring's centre
    for w in ws:
        g = w.gen
        n = _unit(np.cross(g.edge_u[0], g.edge_v[0]))
        assert math.isclose(math.degrees(math.acos(n[2])), 12.0, abs_tol=1e-9)
        c = g.origin.mean(0)
        assert n[0] * c[0] + n[1] * c[1] < 0.0
    # no two generators overlap: their horizontal footprints are disjoint boxes in the ring frame
    ctr = np.array([w.gen.origin.mean(0) for w in ws])
    d = np.linalg.norm(ctr[:, None, :2] - ctr[None, :, :2], axis=-1) + np.eye(88) * 1e9
    width = 4 * W.MOD_W + 3 * 0.02
    assert d.min() > width


def test_own_modules_in_the_scene_act_as_added_occluders(oracle_lib):
    """A generator with its modules among the scene triangles gives the same depth
    pictures and counts as the same generator adding them itself to a scene without them."""
    ws = W.c7_stadium_small()
    for i in (0, 3, 7):
        w = ws[i]
        n2 = 2 * w.gen.n_mod
        keep = np.ones(w.scene.n_tri, bool)
        keep[n2 * i: n2 * (i + 1)] = False
        scene = W.Scene(w.scene.xyz, np.ascontiguousarray(w.scene.tri[keep]))
        g_self = dataclasses.replace(w.gen, add_as_occluders=True)
        a = oracle_lib.evaluate(w.scene, w.gen, w.sweep, w.map_n, w.k, export_maps=True)
        b = oracle_lib.evaluate(scene, g_self, w.sweep, w.map_n, w.k, export_maps=True)
        assert np.array_equal(a.maps, b.maps) and np.array_equal(a.counts, b.counts)
        assert np.array_equal(a.power, b.power)


def test_stadium_shadows_agree_with_ray_casting_outside_band(oracle_lib):
    ws = W.c7_stadium_small()
    sw = ws[0].sweep
    suns = np.arange(0, sw.n, 5)
    sc = ws[0].scene
    tris = sc.xyz[sc.tri]
    shaded = tot = dis = 0
    for i, w in enumerate(ws):
        n2 = 2 * w.gen.n_mod
        others = np.ones(sc.n_tri, bool)
        others[n2 * i: n2 * (i + 1)] = False                 # own modules are coplanar: they never shade
        T = tris[others]
        sub = W.Workload(w.name, w.scene, w.gen, sw.subset(suns), w.map_n, w.k)
        r = oracle_lib.evaluate(sub.scene, sub.gen, sub.sweep, sub.map_n, sub.k, export_bits=True)
        assert r.outside == 0
        pts = G.sample_points(w.gen, w.k).reshape(w.gen.n_mod, -1, 3)
        for j in range(sub.sweep.n):
            s = sub.sweep.sun_xyz[j]
            bits = G.unpack_bits(r.bits[j], w.k).reshape(w.gen.n_mod, -1)
            n = _unit(np.cross(w.gen.edge_u[0], w.gen.edge_v[0]))
            if n @ s <= 0.0:
                assert not bits.any(), "back-lit modules are not tested"
                continue
            vw = oracle_lib.view(w.scene, w.gen, s, w.map_n)
            e1, e2 = vw["e1"], vw["e2"]
            tx, ty = 1.0 / vw["itx"], 1.0 / vw["ity"]
            delta = 0.5 * math.hypot(tx, ty) + 2.0 ** -8 * max(tx, ty) + 1e-9
            P = pts.reshape(-1, 3)
            exact = np.isfinite(G.ray_hits(P, s, T)).any(axis=1)
            got = bits.reshape(-1)
            shaded += int(exact.sum())
            tot += got.size
            bad = np.nonzero(got != exact)[0]
            dis += bad.size
            if bad.size == 0:
                continue
            pu, pv = P[bad] @ e1, P[bad] @ e2
            Tu, Tv = T @ e1, T @ e2
            near_edge = np.zeros(bad.size, bool)
            for a_, b_ in ((0, 1), (1, 2), (2, 0)):
                dist = G.seg_dist(np.stack([pu, pv], 1), np.stack([Tu[:, a_], Tv[:, a_]], 1),
                                  np.stack([Tu[:, b_], Tv[:, b_]], 1))
                near_edge |= (dist <= delta).any(axis=1)
            assert near_edge.all(), f"generator {i} sun {suns[j]}: {(~near_edge).sum()} disagreements off the outline"
    assert shaded > 1000, "the stadium must shade itself on some suns"
    assert dis / tot < 0.02
