"""Pin of the depth origin and scale of the oracle's depth picture (CPU only).

The depth picture (Sec. 2 Step 3, Fig. 3) stores, per pixel, how far the
nearest surface lies from the sun. Its origin (the near side of the scene's
bounding sphere) and its scale (2^24 - 1 units over the range up to the
generator's farthest corner) set every stored value, so a mistake there
changes every exported byte without moving any shadow. The expected values
come from tests/golden/depth_origin.txt, where each one is worked out by hand
from the geometry of two small scenes.
"""
import os

import numpy as np

from paper_1410_5780_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "depth_origin.txt")


def golden():
    out = {}
    for line in open(GOLDEN):
        line = line.strip()
        if line and not line.startswith("#"):
            case, key, val = line.split()
            out[(case, key)] = int(val)
    return out


def _quad(c0, c1, c2, c3):
    return [np.array([c0, c1, c2]), np.array([c0, c2, c3])]


def _flat_module():
    """One horizontal 2 x 2 m module centred on the origin, facing up, 2 x 2 cells."""
    return W.Generator(origin=np.array([[-1.0, -1.0, 0.0]]), edge_u=np.array([[2.0, 0.0, 0.0]]),
                       edge_v=np.array([[0.0, 2.0, 0.0]]), n_cu=2, n_cv=2,
                       cell_substring=np.zeros(4, np.int32), n_sub=1,
                       module_string=np.zeros(1, np.int32), add_as_occluders=True)


def _scene(tris):
    xyz = np.concatenate(tris).reshape(-1, 3).astype(np.float64)
    return W.Scene(xyz, np.arange(xyz.shape[0], dtype=np.int32).reshape(-1, 3))


def _sweep(s):
    s = np.asarray(s, np.float64).reshape(1, 3)
    return W.Sweep(s, np.array([1000.0]), np.array([0.0]), np.array([1.0]), np.array([1], np.int32),
                   np.array([12.0]))


def _picture(oracle_lib, tris, sun, n):
    r = oracle_lib.evaluate(_scene(tris), _flat_module(), _sweep(sun), n, 2, export_maps=True)
    assert r.outside == 0
    return r.maps[0].astype(np.int64)


def test_zenith_depths_of_horizontal_planes(oracle_lib):
    """Sun at the zenith: a horizontal plane at height h lies at (c_z + R - h) Dmax / (c_z + R)
    with c_z = 1 and R = 3 for this scene; exact in binary64, so the picture must match exactly."""
    g = golden()
    tris = (_quad((-2.0, -2.0, 2.0), (0.0, -2.0, 2.0), (0.0, 2.0, 2.0), (-2.0, 2.0, 2.0))
            + _quad((0.0, -2.0, 1.0), (2.0, -2.0, 1.0), (2.0, 2.0, 1.0), (0.0, 2.0, 1.0)))
    pic = _picture(oracle_lib, tris, (0.0, 0.0, 1.0), 16)
    want = np.empty((16, 16), np.int64)
    want[:8, :] = g[("zenith", "rows_below_half")]
    want[8:, :] = g[("zenith", "rows_above_half")]
    assert np.array_equal(pic, want), f"rows {np.unique(pic, axis=1)[:, 0].tolist()}"


def test_oblique_depths_of_planes_facing_the_sun(oracle_lib):
    """Sun (0, -0.6, 0.8): two squares perpendicular to the sun at depths t = -2.5 and -1.5,
    over a scene box whose sphere is c = (0, -2, 2), R = 6 (two marker triangles far outside
    the window fix the box). Depth (t - z_near) Dmax / 9.4 with z_near = -8.8, within one unit."""
    g = golden()
    s = np.array([0.0, -0.6, 0.8])
    d = -s
    e1, e2 = np.array([-1.0, 0.0, 0.0]), np.array([0.0, 0.8, 0.6])

    def square(t, a0, a1):
        q = t * d
        c = [q + a * e1 + b * e2 for a, b in ((a0, -2.0), (a1, -2.0), (a1, 2.0), (a0, 2.0))]
        return _quad(*c)

    markers = [np.array([(-4.0, -6.0, 0.0), (-3.9, -6.0, 0.0), (-4.0, -5.9, 0.0)]),
               np.array([(4.0, 2.0, 4.0), (3.9, 2.0, 4.0), (4.0, 1.9, 4.0)])]
    tris = square(-2.5, 0.0, 2.0) + square(-1.5, -2.0, 0.0) + markers
    lo = np.concatenate(tris).min(axis=0)
    hi = np.concatenate(tris).max(axis=0)
    assert np.allclose(lo, (-4, -6, 0)) and np.allclose(hi, (4, 2, 4))     # the box of the derivation
    pic = _picture(oracle_lib, tris, s, 18)
    right, left = g[("oblique", "cols_right")], g[("oblique", "cols_left")]
    assert np.all(np.abs(pic[:, 9:] - right) <= 1), np.unique(pic[:, 9:]).tolist()
    assert np.all(np.abs(pic[:, :9] - left) <= 1), np.unique(pic[:, :9]).tolist()
    # the depth scale alone: the two planes lie 1 m apart along the view axis
    gap = int(np.median(pic[:, :9])) - int(np.median(pic[:, 9:]))
    assert abs(gap - (left - right)) <= 1 and abs(gap - 16777215 / 9.4) <= 2
