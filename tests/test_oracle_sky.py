"""Pins of the oracle's diffuse shading (sky view factors), CPU only.

A cell's sky view factor is the cosine-weighted share of the sky in front of
its module that it sees, over a fixed set of directions standing for equal
solid angles. Checked here: a generator with nothing around it sees the whole
sky exactly; beside a long wall, the factor matches the closed form of the
cosine-weighted view past an infinite wall, for horizontal and for tilted
receivers, with the wall in front and behind (within the quadrature error of
4,096 directions); an added occluder never raises it; the direction set covers
equal solid angles; and the factor scales only the diffuse, while the
reference power keeps the whole sky.
"""
import dataclasses
import math

import numpy as np
import pytest

from paper_1410_5780_amd import workloads as W
from tests import _geom as G

N_DIR = 4096


def test_sky_directions_cover_equal_solid_angles():
    d = W.sky_directions(N_DIR)
    assert np.allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-15) and np.all(d[:, 2] > 0)
    # Archimedes: equal bands of height hold equal solid angle, so heights are uniform on (0, 1)
    assert np.mean(d[:, 2]) == pytest.approx(0.5, abs=1e-12)
    assert np.mean(d[:, 2] ** 2) == pytest.approx(1.0 / 3.0, abs=1e-6)
    # azimuths spread evenly: the mean horizontal direction nearly vanishes
    assert np.linalg.norm(d[:, :2].mean(0)) < 1e-3


def _flat_gen(tilt_deg=0.0, n_side=2):
    """n_side x n_side portrait modules around the origin, tilted toward the south by tilt_deg."""
    b = math.radians(tilt_deg)
    u = np.array([W.MOD_W, 0.0, 0.0])
    v = W.MOD_L * np.array([0.0, math.cos(b), math.sin(b)])
    o = np.array([[-W.MOD_W + i * (W.MOD_W + 0.02), -W.MOD_L + j * (W.MOD_L + 0.02), 0.5] for i in range(n_side)
                  for j in range(n_side)])
    o[:, 1] = o[:, 1] * math.cos(b)
    o[:, 2] = 0.5 + (o[:, 1] + W.MOD_L * math.cos(b)) * math.tan(b) if tilt_deg else 0.5
    m = o.shape[0]
    return W.Generator(o, np.tile(u, (m, 1)), np.tile(v, (m, 1)), W.N_CU, W.N_CV, W.portrait_substrings(), 3,
                       np.zeros(m, np.int32), add_as_occluders=False)


def _wall(y_face, height, north=True, length=600.0, thick=0.2):
    m = W._Mesh()
    cy = y_face + (thick / 2 if north else -thick / 2)
    m.add(*W.boxes(np.array([0.0]), np.array([cy]), length, thick, 0.0, height, 0.0, floor=False))
    return m.scene()


def _sample_alpha(g, k, y_face, height, north):
    pts = G.sample_points(g, k).reshape(g.n_mod * g.n_cv * g.n_cu, k * k, 3)
    dist = (y_face - pts[..., 1]) if north else (pts[..., 1] - y_face)
    return np.arctan2(height - pts[..., 2], dist)


def test_lone_generator_sees_the_whole_sky(oracle_lib):
    for tilt in (0.0, 30.0, 75.0):
        g = _flat_gen(tilt)
        svf = oracle_lib.sky_view(W.Scene(np.zeros((0, 3)), np.zeros((0, 3), np.int32)), g, W.sky_directions(512),
                                  128, 2)
        assert np.all(svf == 1.0)


@pytest.mark.parametrize("tilt,north", [(0.0, True), (30.0, True), (30.0, False)])
def test_wall_matches_the_infinite_wall_closed_form(oracle_lib, tilt, north):
    """Cosine-weighted view past an infinite wall whose top stands at elevation a, for a
    receiver tilted b toward the south (front sky: (1 + cos b) / 2 of the hemisphere):
      wall to the north (behind): 1 - (1 - cos(a - b)) / (1 + cos b), nothing hidden when a <= b;
      wall to the south (in front): 1 - (cos b - cos(a + b)) / (1 + cos b)."""
    g = _flat_gen(tilt)
    k = 2
    y_face, height = (4.0, 6.0) if north else (-4.0, 3.0)
    sc = _wall(y_face, height, north)
    svf = oracle_lib.sky_view(sc, g, W.sky_directions(N_DIR), 256, k)
    a = _sample_alpha(g, k, y_face, height, north)
    b = math.radians(tilt)
    if north:
        hidden = np.where(a > b, (1.0 - np.cos(a - b)), 0.0) / (1.0 + math.cos(b))
    else:
        hidden = (math.cos(b) - np.cos(a + b)) / (1.0 + math.cos(b))
    want = (1.0 - hidden).mean(axis=1)
    assert np.abs(svf - want).max() < 2.5e-3, (np.abs(svf - want).max(), svf.min(), want.min())
    assert want.min() < 0.97, "the wall must hide a fair share of the sky"


def test_added_occluder_never_raises_the_view(oracle_lib):
    w = W.c1_tiny()
    g = w.gen
    d = W.sky_directions(1024)
    with_pole = oracle_lib.sky_view(w.scene, g, d, 256, 4)
    alone = oracle_lib.sky_view(W.Scene(np.zeros((0, 3)), np.zeros((0, 3), np.int32)), g, d, 256, 4)
    assert np.all(alone == 1.0) and np.all(with_pole <= 1.0) and with_pole.min() < 0.99
    m = W._Mesh()
    m.add(w.scene.xyz[w.scene.tri], np.array([[0, 1, 2]]))
    m.add(*W.boxes(np.array([-3.0]), np.array([1.5]), 1.0, 1.0, 0.0, 3.0, 0.0, floor=False))
    more = oracle_lib.sky_view(m.scene(), g, d, 256, 4)
    assert np.all(more <= with_pole + 1e-15) and more.min() < with_pole.min()


def test_sky_view_scales_only_the_diffuse(oracle_lib):
    """With no beam, a lone module's cells get d_poa * svf: the ideal string power is that of
    the substrings' weakest cells, and the reference keeps the whole sky."""
    w = W.c1_tiny(d_poa=100.0)
    sw = dataclasses.replace(w.sweep, dni=np.zeros(w.sweep.n))
    rng = np.random.default_rng(5)
    svf = rng.uniform(0.3, 1.0, w.gen.n_cells)
    g = dataclasses.replace(w.gen, sky_view=svf)
    empty = W.Scene(np.zeros((0, 3)), np.zeros((0, 3), np.int32))
    r = oracle_lib.evaluate(empty, g, sw, w.map_n, w.k)
    up = sw.sun_xyz[:, 2] > 0
    caps = [100.0 * svf[g.cell_substring == q].min() for q in range(3)]
    want = max((j + 1) * c for j, c in enumerate(sorted(caps, reverse=True)))
    np.testing.assert_allclose(r.power[up], want, rtol=1e-15)
    np.testing.assert_allclose(r.power_ref[up], 300.0, rtol=1e-15)
    # the diode model takes the cells' diffuse shares too
    gd = dataclasses.replace(g, diode=W.DIODE_CELL)
    rd = oracle_lib.evaluate(empty, gd, sw, w.map_n, w.k)
    subs = [list(100.0 * svf[g.cell_substring == q]) for q in range(3)]
    gg = np.concatenate([np.asarray(s) for s in subs])
    assert rd.power[up][0] == pytest.approx(oracle_lib.string_mpp(W.DIODE_CELL, gg, [20, 20, 20]), rel=1e-12)
    assert np.all(rd.power[up] < rd.power_ref[up])
