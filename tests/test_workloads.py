"""Pins of the input generators (sun positions and scene shapes), CPU only."""
import math

import numpy as np
import pytest

from paper_1410_5780_amd import workloads as W

PHI = 40.4


def _noon_declination(day):
    # at solar noon the sun lies in the meridian plane: elevation = 90 - (phi - delta)
    s = W.cooper_sun(PHI, [day], [12.0])[0]
    assert abs(s[0]) < 1e-15
    return PHI + math.degrees(math.atan2(s[1], s[2]))


def test_cooper_declination_extremes():
    # Cooper: 23.45 sin(360 (284 + n) / 365); day 355 is the winter, 172 the summer extreme
    assert _noon_declination(355) == pytest.approx(-23.449783, abs=1e-6)
    assert _noon_declination(172) == pytest.approx(23.449783, abs=1e-6)
    assert _noon_declination(81) == pytest.approx(0.0, abs=1e-12)
    assert _noon_declination(1) == pytest.approx(-23.011637, abs=1e-6)


def test_sun_vectors_unit_and_elevations_day355():
    s = W.cooper_sun(PHI, np.full(24, 355), np.arange(24.0))
    assert np.all(np.abs(np.linalg.norm(s, axis=1) - 1.0) < 1e-12)
    elev = np.degrees(np.arcsin(s[:, 2]))
    up = np.nonzero(s[:, 2] > 0)[0]
    assert list(up) == list(range(8, 17))
    want = [5.244, 13.656, 20.312, 24.640, 26.150, 24.640, 20.312, 13.656, 5.244]
    assert np.allclose(elev[8:17], want, atol=1e-3)
    # morning sun in the east (x > 0), afternoon in the west, symmetric about noon
    assert np.all(s[8:12, 0] > 0) and np.all(s[13:17, 0] < 0)
    assert np.allclose(s[8:12, [1, 2]], s[16:12:-1, [1, 2]], atol=1e-14)


def test_year_up_hours_match_sunrise_hour_angle():
    """Count of hourly suns above the horizon vs the sunrise hour angle acos(-tan phi tan delta)."""
    yr = W.make_sweep(PHI, np.arange(1, 366), np.arange(24.0))
    z = yr.sun_xyz[:, 2]
    phi = math.radians(PHI)
    n_up_formula = 0
    boundary = 0
    for day in range(1, 366):
        d = math.radians(23.45 * math.sin(math.radians(360.0 * (284 + day) / 365.0)))
        ws = math.degrees(math.acos(-math.tan(phi) * math.tan(d)))
        for h in range(24):
            w = abs(15.0 * (h - 12))
            if abs(w - ws) < 1e-9:
                boundary += 1
            elif w < ws:
                n_up_formula += 1
    near = np.abs(z) < 1e-12
    assert boundary == near.sum() == 2            # equinox sunrise / sunset sit on the horizon
    assert int(((z > 0) & ~near).sum()) == n_up_formula == 4379
    assert W.year_sweep().n == 4379
    # day length on day 355: 2 ws / 15 = 9.1114 h
    d = math.radians(23.45 * math.sin(math.radians(360.0 * (284 + 355) / 365.0)))
    assert 2 * math.degrees(math.acos(-math.tan(phi) * math.tan(d))) / 15 == pytest.approx(9.1114, abs=1e-4)


def test_config_sizes():
    c1 = W.c1_tiny()
    assert (c1.scene.n_tri, c1.n_tri_submitted, c1.gen.n_cells, c1.n_samples) == (12, 14, 60, 15360)
    c2 = W.c2_row_plant(sweep=W.make_sweep(PHI, [355], [12.0]))
    assert c2.n_tri_submitted == 101602 and c2.scene.n_vert == 67204 and c2.gen.n_cells == 24000
    assert c2.n_samples == 1536000
    c3 = W.c3_rooftop(sweep=W.make_sweep(PHI, [355], [12.0]))
    assert c3.n_tri_submitted == 522010 and c3.gen.n_cells == 120000 and c3.n_samples == 7680000
    # module geometry: 156 mm cells, portrait 6 x 10, 30 deg tilt facing south
    u, v = c1.gen.edge_u[0], c1.gen.edge_v[0]
    assert np.linalg.norm(u) == pytest.approx(0.936) and np.linalg.norm(v) == pytest.approx(1.56)
    n = np.cross(u, v) / np.linalg.norm(np.cross(u, v))
    assert np.allclose(n, [0, -0.5, math.sqrt(3) / 2])
    assert list(c1.gen.cell_substring[:6]) == [0, 0, 1, 1, 2, 2]


def test_generators_deterministic():
    a = W.c2_row_plant(seed=2, sweep=W.make_sweep(PHI, [1], [12.0]))
    b = W.c2_row_plant(seed=2, sweep=W.make_sweep(PHI, [1], [12.0]))
    assert np.array_equal(a.scene.xyz, b.scene.xyz) and np.array_equal(a.scene.tri, b.scene.tri)
    t = W.random_tiny(7)
    assert t.scene.tri.max() < t.scene.n_vert


def test_icosphere_and_pylon_counts():
    v, t = W.icosphere(5)
    assert v.shape == (252, 3) and t.shape == (500, 3)
    assert np.allclose(np.linalg.norm(v, axis=1), 1.0)
    pv, pt = W.pylons([0.0], [0.0], [0.3])
    assert pv.shape == (1, 1344, 3) and pt.shape == (2016, 3)
    assert pv[..., 2].max() <= 30.0 + 0.1
