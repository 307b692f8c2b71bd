"""Seeded synthetic inputs for the shadow-map shading path.

This module only *builds inputs*: triangle scenes, PV generator tables and sun
sweeps. It holds none of the method's arithmetic (no light-space transform, no
raster, no depth test, no loss model), so the oracle and the HIP path can both
consume what it produces without sharing any computation.

The paper's scenes (Google Earth / 3D Warehouse models of a house, tree and
streetlight in Sec. 3.1, a tracker plant with an electrical pylon in Sec. 3.4)
are not available; the generators here produce scenes of the same kind and
size: lattice pylons, box buildings, icosphere trees, module rows and roofs.

Sun positions follow Cooper's declination and a 15 deg/h hour angle: the
paper only states that the solar position is defined for a date, time and
location (Sec. 2, Step 3), so the sweep is an input to the path.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

CELL = 0.156            # PV cell edge, metres
N_CU, N_CV = 6, 10      # portrait 60-cell module: 6 cells across, 10 along the slope
MOD_W = N_CU * CELL     # 0.936 m
MOD_L = N_CV * CELL     # 1.56 m
LAT_DEG = 40.4

# A 156 mm monocrystalline cell at 25 C for the single-diode model: Isc 9.0 A at
# 1000 W/m^2, open-circuit voltage about 0.63 V (ideality 1.2, kT/q 25.693 mV),
# Rs 4 mOhm, Rsh 15 Ohm; Schottky bypass diodes at 0.4 V.
DIODE_CELL = np.array([9.0, 1000.0, 1.2e-8, 1.2 * 0.025693, 0.004, 15.0, 0.4])


# --------------------------------------------------------------------------
# containers
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Scene:
    """Triangle soup in ENU metres (x east, y north, z up)."""
    xyz: np.ndarray        # float64 [V, 3]
    tri: np.ndarray        # int32 [T, 3]

    @property
    def n_vert(self) -> int:
        return int(self.xyz.shape[0])

    @property
    def n_tri(self) -> int:
        return int(self.tri.shape[0])


@dataclasses.dataclass
class Generator:
    """PV generator: rectangular modules split into n_cu x n_cv cells.

    Module m spans origin + a*edge_u + b*edge_v for a, b in [0, 1]; its front
    face is the side edge_u x edge_v points to. Cell (cu, cv) has index
    cv*n_cu + cu; ``cell_substring`` maps that index to the module's bypass
    substring; ``module_string`` gives each module's series string.
    """
    origin: np.ndarray         # float64 [M, 3]
    edge_u: np.ndarray         # float64 [M, 3]
    edge_v: np.ndarray         # float64 [M, 3]
    n_cu: int
    n_cv: int
    cell_substring: np.ndarray  # int32 [n_cu*n_cv]
    n_sub: int
    module_string: np.ndarray  # int32 [M]
    add_as_occluders: bool = True
    # trackers: modules given at rest, turned about a pivot as the sun moves
    # (None: the modules stay put). trackers [T, 7] = kind (1 one horizontal
    # axis, 2 two axes), pivot xyz, horizontal unit axis xyz; module_tracker
    # [M] the tracker of each module, -1 for none.
    trackers: Optional[np.ndarray] = None
    module_tracker: Optional[np.ndarray] = None
    # electrical model: None for ideal bypass-diode strings, else the single-diode
    # cell parameters [7] = Isc_ref (A), G_ref (W/m^2), I0 (A), a = n k T / q (V),
    # Rs (ohm), Rsh (ohm) and the bypass diode's forward voltage Vb (V)
    diode: Optional[np.ndarray] = None
    # diffuse shading: per-cell sky view factors [n_cells] in [0, 1] scaling the
    # diffuse irradiance (None: every cell sees the whole sky)
    sky_view: Optional[np.ndarray] = None

    @property
    def n_mod(self) -> int:
        return int(self.origin.shape[0])

    @property
    def n_cells(self) -> int:
        return self.n_mod * self.n_cu * self.n_cv

    @property
    def n_string(self) -> int:
        return int(self.module_string.max()) + 1 if self.n_mod else 0


@dataclasses.dataclass
class Sweep:
    """Sun positions and the irradiance that goes with them."""
    sun_xyz: np.ndarray   # float64 [n, 3] unit vectors toward the sun (ENU)
    dni: np.ndarray       # float64 [n] W/m^2, direct normal irradiance
    d_poa: np.ndarray     # float64 [n] W/m^2, diffuse on the plane of array
    dt_h: np.ndarray      # float64 [n] hours represented by each sun
    day: np.ndarray       # int32 [n]
    hour: np.ndarray      # float64 [n]

    @property
    def n(self) -> int:
        return int(self.sun_xyz.shape[0])

    def subset(self, idx) -> "Sweep":
        idx = np.asarray(idx)
        return Sweep(self.sun_xyz[idx].copy(), self.dni[idx].copy(), self.d_poa[idx].copy(),
                     self.dt_h[idx].copy(), self.day[idx].copy(), self.hour[idx].copy())


@dataclasses.dataclass
class Workload:
    name: str
    scene: Scene
    gen: Generator
    sweep: Sweep
    map_n: int
    k: int
    note: str = ""

    @property
    def n_samples(self) -> int:
        return self.gen.n_cells * self.k * self.k

    @property
    def n_tri_submitted(self) -> int:
        return self.scene.n_tri + (2 * self.gen.n_mod if self.gen.add_as_occluders else 0)


# --------------------------------------------------------------------------
# sun positions (input side)
# --------------------------------------------------------------------------
def cooper_sun(lat_deg: float, day, hour) -> np.ndarray:
    """Unit vectors toward the sun in ENU for day-of-year and local solar hour.

    Declination after Cooper: 23.45 deg * sin(360 deg * (284 + n) / 365);
    hour angle 15 deg per hour from solar noon; no equation of time,
    longitude correction or refraction.
    """
    day = np.asarray(day, dtype=np.float64)
    hour = np.asarray(hour, dtype=np.float64)
    decl = np.deg2rad(23.45 * np.sin(np.deg2rad(360.0 * (284.0 + day) / 365.0)))
    omega = np.deg2rad(15.0 * (hour - 12.0))
    phi = math.radians(lat_deg)
    cd, sd = np.cos(decl), np.sin(decl)
    sx = -cd * np.sin(omega)
    sy = sd * math.cos(phi) - cd * math.sin(phi) * np.cos(omega)
    sz = sd * math.sin(phi) + cd * math.cos(phi) * np.cos(omega)
    return np.stack([sx, sy, sz], axis=-1)


def make_sweep(lat_deg: float, days, hours, dni=1000.0, d_poa=100.0, dt_h=1.0,
               up_only: bool = False) -> Sweep:
    days = np.asarray(days, dtype=np.int32)
    hours = np.asarray(hours, dtype=np.float64)
    dd, hh = np.meshgrid(days, hours, indexing="ij")
    dd, hh = dd.ravel(), hh.ravel()
    s = cooper_sun(lat_deg, dd, hh)
    if up_only:
        keep = s[:, 2] > 0.0
        s, dd, hh = s[keep], dd[keep], hh[keep]
    n = s.shape[0]
    return Sweep(np.ascontiguousarray(s), np.full(n, float(dni)), np.full(n, float(d_poa)),
                 np.full(n, float(dt_h)), dd.astype(np.int32), hh.astype(np.float64))


def year_sweep(lat_deg: float = LAT_DEG, step_min: int = 60, dni=1000.0, d_poa=100.0) -> Sweep:
    """All suns strictly above the horizon in a year (hourly at 40.4 N: 4,379)."""
    hours = np.arange(0, 24 * 60, step_min, dtype=np.float64) / 60.0
    return make_sweep(lat_deg, np.arange(1, 366), hours, dni=dni, d_poa=d_poa,
                      dt_h=step_min / 60.0, up_only=True)


# --------------------------------------------------------------------------
# mesh pieces
# --------------------------------------------------------------------------
class _Mesh:
    def __init__(self):
        self.v: List[np.ndarray] = []
        self.t: List[np.ndarray] = []
        self.nv = 0

    def add(self, v: np.ndarray, t: np.ndarray):
        """Append a batch: v [..., nv, 3], t [nt, 3] template indices (same per item)."""
        v = np.asarray(v, dtype=np.float64)
        if v.ndim == 2:
            v = v[None]
        nb, nvi = v.shape[0], v.shape[1]
        off = self.nv + nvi * np.arange(nb, dtype=np.int64)[:, None, None]
        self.v.append(v.reshape(-1, 3))
        self.t.append((np.asarray(t, dtype=np.int64)[None] + off).reshape(-1, 3))
        self.nv += nb * nvi

    def scene(self) -> Scene:
        if not self.v:
            return Scene(np.zeros((0, 3)), np.zeros((0, 3), dtype=np.int32))
        xyz = np.ascontiguousarray(np.concatenate(self.v, 0))
        tri = np.concatenate(self.t, 0)
        assert tri.max() < 2 ** 31
        return Scene(xyz, np.ascontiguousarray(tri.astype(np.int32)))


_BOX_T = np.array([[0, 2, 1], [0, 3, 2],                      # bottom
                   [4, 5, 6], [4, 6, 7],                      # top
                   [0, 1, 5], [0, 5, 4], [1, 2, 6], [1, 6, 5],
                   [2, 3, 7], [2, 7, 6], [3, 0, 4], [3, 4, 7]], dtype=np.int64)
_BOX_T_NOFLOOR = _BOX_T[2:]


def _rotz(yaw):
    c, s = np.cos(yaw), np.sin(yaw)
    return c, s


def boxes(cx, cy, sx, sy, z0, z1, yaw, floor: bool = True):
    """Batch of yawed boxes. Returns (verts [n,8,3], tri template)."""
    cx, cy, sx, sy, z0, z1, yaw = (np.atleast_1d(np.asarray(a, dtype=np.float64))
                                   for a in (cx, cy, sx, sy, z0, z1, yaw))
    n = max(len(cx), len(cy), len(sx), len(sy), len(z0), len(z1), len(yaw))
    bx = np.array([-0.5, 0.5, 0.5, -0.5])
    by = np.array([-0.5, -0.5, 0.5, 0.5])
    lx = bx[None] * np.broadcast_to(sx, (n,))[:, None]
    ly = by[None] * np.broadcast_to(sy, (n,))[:, None]
    c, s = _rotz(np.broadcast_to(yaw, (n,)))
    gx = np.broadcast_to(cx, (n,))[:, None] + c[:, None] * lx - s[:, None] * ly
    gy = np.broadcast_to(cy, (n,))[:, None] + s[:, None] * lx + c[:, None] * ly
    v = np.empty((n, 8, 3))
    v[:, :4, 0] = gx
    v[:, :4, 1] = gy
    v[:, :4, 2] = np.broadcast_to(z0, (n,))[:, None]
    v[:, 4:, 0] = gx
    v[:, 4:, 1] = gy
    v[:, 4:, 2] = np.broadcast_to(z1, (n,))[:, None]
    return v, (_BOX_T if floor else _BOX_T_NOFLOOR)


def beam_vertices(p: np.ndarray, q: np.ndarray, width: float) -> np.ndarray:
    """Square-section beams from p to q: p, q [n,3] -> vertices [n,8,3] (box topology)."""
    p = np.asarray(p, dtype=np.float64)
    q = np.asarray(q, dtype=np.float64)
    t = q - p
    t = t / np.linalg.norm(t, axis=1, keepdims=True)
    a = np.where(np.abs(t[:, 2:3]) < 0.9, np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]]))
    u = np.cross(a, t)
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    w = np.cross(t, u)
    h = 0.5 * width
    off = np.stack([-u - w, u - w, u + w, -u + w], axis=1) * h     # [n,4,3]
    v = np.empty((p.shape[0], 8, 3))
    v[:, :4] = p[:, None, :] + off
    v[:, 4:] = q[:, None, :] + off
    return v


def _pylon_template(height=30.0, base_w=6.0, top_w=1.5, panels=10, beam=0.1) -> np.ndarray:
    """One lattice pylon at the origin, yaw 0: 168 beams -> vertices [168*8, 3]."""
    lv = np.arange(panels + 1)
    hw = 0.5 * base_w * (1 - lv / panels) + 0.5 * top_w * (lv / panels)
    z = height * lv / panels
    sgn = np.array([[-1, -1], [1, -1], [1, 1], [-1, 1]], dtype=np.float64)

    def corner(l, c):
        return np.array([sgn[c % 4, 0] * hw[l], sgn[c % 4, 1] * hw[l], z[l]])

    P, Q = [], []
    for l in range(panels):                       # legs
        for c in range(4):
            P.append(corner(l, c)); Q.append(corner(l + 1, c))
    for l in range(1, panels + 1):                # horizontal struts
        for c in range(4):
            P.append(corner(l, c)); Q.append(corner(l, c + 1))
    for l in range(panels):                       # X-bracing on every face
        for c in range(4):
            P.append(corner(l, c)); Q.append(corner(l + 1, c + 1))
            P.append(corner(l, c + 1)); Q.append(corner(l + 1, c))
    za, zb = z[8], z[9]                           # cross-arms
    tips = [np.array([-5.0, 0, za]), np.array([5.0, 0, za]), np.array([-4.0, 0, zb]), np.array([4.0, 0, zb])]
    P += [tips[0], tips[2]]; Q += [tips[1], tips[3]]
    P += [tips[0], tips[1]]; Q += [corner(7, 0), corner(7, 1)]
    P += [tips[2], tips[3]]; Q += [corner(8, 3), corner(8, 2)]
    P += [tips[0], tips[1]]; Q += [tips[2], tips[3]]
    P, Q = np.array(P), np.array(Q)
    assert P.shape[0] == 168
    return beam_vertices(P, Q, beam).reshape(-1, 3)


_PYLON = None


def pylons(cx, cy, yaw):
    """Batch of 2,016-triangle lattice pylons (30 m tall, 6 m base, 1.5 m top)."""
    global _PYLON
    if _PYLON is None:
        _PYLON = _pylon_template()
    cx, cy, yaw = (np.atleast_1d(np.asarray(a, dtype=np.float64)) for a in (cx, cy, yaw))
    c, s = _rotz(yaw)
    t = _PYLON
    v = np.empty((len(cx), t.shape[0], 3))
    v[..., 0] = cx[:, None] + c[:, None] * t[None, :, 0] - s[:, None] * t[None, :, 1]
    v[..., 1] = cy[:, None] + s[:, None] * t[None, :, 0] + c[:, None] * t[None, :, 1]
    v[..., 2] = t[None, :, 2]
    tri = (np.arange(168)[:, None, None] * 8 + _BOX_T[None]).reshape(-1, 3)
    return v, tri


def icosphere(freq: int = 5):
    """Geodesic icosphere: 10 f^2 + 2 vertices, 20 f^2 triangles on the unit sphere."""
    g = (1 + 5 ** 0.5) / 2
    V = np.array([[-1, g, 0], [1, g, 0], [-1, -g, 0], [1, -g, 0], [0, -1, g], [0, 1, g],
                  [0, -1, -g], [0, 1, -g], [g, 0, -1], [g, 0, 1], [-g, 0, -1], [-g, 0, 1]], float)
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
         (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
         (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    key = {}
    verts = []

    def vid(p):
        p = p / np.linalg.norm(p)
        kk = tuple(np.round(p, 9))
        if kk not in key:
            key[kk] = len(verts)
            verts.append(p)
        return key[kk]

    tris = []
    for a, b, c in F:
        A, B, C = V[a], V[b], V[c]
        idx = {}
        for i in range(freq + 1):
            for j in range(freq + 1 - i):
                idx[(i, j)] = vid(A + (B - A) * i / freq + (C - A) * j / freq)
        for i in range(freq):
            for j in range(freq - i):
                tris.append((idx[(i, j)], idx[(i + 1, j)], idx[(i, j + 1)]))
                if i + j < freq - 1:
                    tris.append((idx[(i + 1, j)], idx[(i + 1, j + 1)], idx[(i, j + 1)]))
    return np.array(verts), np.array(tris, dtype=np.int64)


_TREE = None


def _tree_template():
    """Unit tree (crown radius 1): 8-sided open trunk (16 tris) + frequency-5 crown (500 tris)."""
    sv, st = icosphere(5)
    ang = 2 * np.pi * np.arange(8) / 8
    tr = 0.1
    trunk = np.concatenate([np.stack([tr * np.cos(ang), tr * np.sin(ang), np.zeros(8)], 1),
                            np.stack([tr * np.cos(ang), tr * np.sin(ang), np.full(8, 2.0)], 1)])
    tt = []
    for i in range(8):
        j = (i + 1) % 8
        tt += [(i, j, 8 + j), (i, 8 + j, 8 + i)]
    crown = sv + np.array([0.0, 0.0, 2.7])
    v = np.concatenate([trunk, crown])
    t = np.concatenate([np.array(tt), st + 16])
    return v, t


def trees(cx, cy, r):
    global _TREE
    if _TREE is None:
        _TREE = _tree_template()
    tv, tt = _TREE
    cx, cy, r = (np.atleast_1d(np.asarray(a, dtype=np.float64)) for a in (cx, cy, r))
    v = tv[None] * r[:, None, None]
    v[..., 0] += cx[:, None]
    v[..., 1] += cy[:, None]
    return v, tt


def _annulus(rng, n, r0, r1, cx=0.0, cy=0.0):
    rad = np.sqrt(rng.uniform(r0 * r0, r1 * r1, n))
    th = rng.uniform(0, 2 * np.pi, n)
    return cx + rad * np.cos(th), cy + rad * np.sin(th)


# --------------------------------------------------------------------------
# PV generators
# --------------------------------------------------------------------------
def portrait_substrings(n_cu=N_CU, n_cv=N_CV, n_sub=3) -> np.ndarray:
    """Substring s holds cell columns {2s, 2s+1} (10 cells along the slope each)."""
    cu = np.tile(np.arange(n_cu), n_cv)
    return (cu * n_sub // n_cu).astype(np.int32)


def module_rows(n_rows: int, per_row: int, tilt_deg: float = 30.0, pitch: float = 3.9,
                z0: float = 0.5, gap: float = 0.02, x0: float = 0.0, y0: float = 0.0,
                modules_per_string: int = 20, n_mod: Optional[int] = None) -> Generator:
    """South-facing fixed-tilt portrait rows; modules fill rows in order, strings of <= 20."""
    b = math.radians(tilt_deg)
    U = np.array([MOD_W, 0.0, 0.0])
    V = np.array([0.0, MOD_L * math.cos(b), MOD_L * math.sin(b)])
    total = n_rows * per_row if n_mod is None else n_mod
    m = np.arange(total)
    r, c = m // per_row, m % per_row
    O = np.stack([x0 + c * (MOD_W + gap), y0 + r * pitch, np.full(total, z0)], 1)
    ms = (m // modules_per_string).astype(np.int32)
    return Generator(np.ascontiguousarray(O), np.tile(U, (total, 1)), np.tile(V, (total, 1)),
                     N_CU, N_CV, portrait_substrings(), 3, ms)


def ground_plane(x0, y0, x1, y1, z=0.0):
    v = np.array([[x0, y0, z], [x1, y0, z], [x1, y1, z], [x0, y1, z]], float)
    return v, np.array([[0, 1, 2], [0, 2, 3]])


def gen_bbox(gen: Generator):
    c = np.concatenate([gen.origin, gen.origin + gen.edge_u, gen.origin + gen.edge_u + gen.edge_v,
                        gen.origin + gen.edge_v])
    return c.min(0), c.max(0)


# --------------------------------------------------------------------------
# trackers
# --------------------------------------------------------------------------
def tracker_generator(pivots, kind: int, axis=(0.0, 1.0, 0.0), n_u: int = 7, n_v: int = 4,
                      gap: float = 0.02, modules_per_string: int = 14, lift: float = 0.15) -> Generator:
    """Trackers of n_u x n_v portrait modules each, flat and facing up at rest,
    centred over their pivots and `lift` metres above them: the 6-cell side
    runs along u0 = axis x z (n_u modules), the 10-cell side along v0 = axis
    (n_v modules). kind 1 turns about the horizontal axis, kind 2 about two axes."""
    pv = np.atleast_2d(np.asarray(pivots, dtype=np.float64))
    a = np.asarray(axis, dtype=np.float64)
    assert a[2] == 0.0 and abs(np.dot(a, a) - 1.0) < 1e-12, "the axis is a horizontal unit vector"
    u0 = np.array([a[1], -a[0], 0.0])            # a x z
    v0 = a
    w = n_u * MOD_W + (n_u - 1) * gap
    h = n_v * MOD_L + (n_v - 1) * gap
    nt, per = pv.shape[0], n_u * n_v
    m = np.arange(nt * per)
    t, i, j = m // per, (m % per) % n_u, (m % per) // n_u
    au = -w / 2 + i * (MOD_W + gap)
    bv = -h / 2 + j * (MOD_L + gap)
    O = pv[t] + au[:, None] * u0[None] + bv[:, None] * v0[None] + np.array([0.0, 0.0, lift])
    trk = np.concatenate([np.full((nt, 1), float(kind)), pv, np.tile(a, (nt, 1))], 1)
    return Generator(np.ascontiguousarray(O), np.tile(MOD_W * u0, (nt * per, 1)), np.tile(MOD_L * v0, (nt * per, 1)),
                     N_CU, N_CV, portrait_substrings(), 3, (m // modules_per_string).astype(np.int32),
                     trackers=np.ascontiguousarray(trk), module_tracker=t.astype(np.int32))


def terrain(x0, y0, x1, y1, n: int, rng, hills: int = 6, height: float = 3.0, spread: float = 40.0):
    """Uneven ground: an n x n grid of quads over [x0, x1] x [y0, y1], heights a sum of Gaussian hills."""
    cx = rng.uniform(x0, x1, hills)
    cy = rng.uniform(y0, y1, hills)
    amp = rng.uniform(-height, height, hills)
    xs, ys = np.linspace(x0, x1, n + 1), np.linspace(y0, y1, n + 1)
    X, Y = np.meshgrid(xs, ys, indexing="xy")

    def z_at(x, y):
        x, y = np.asarray(x, float), np.asarray(y, float)
        return sum(a * np.exp(-((x - u) ** 2 + (y - v) ** 2) / (2 * spread ** 2)) for a, u, v in zip(amp, cx, cy))

    v = np.stack([X.ravel(), Y.ravel(), z_at(X.ravel(), Y.ravel())], 1)
    q = np.arange(n * n)
    r, c = q // n, q % n
    a0 = r * (n + 1) + c
    t = np.concatenate([np.stack([a0, a0 + 1, a0 + n + 2], 1), np.stack([a0, a0 + n + 2, a0 + n + 1], 1)])
    return v, t, z_at


def tracker_pair(gap_m: float = 4.0, kind: int = 2, map_n: int = 512, k: int = 4,
                 sweep: Optional[Sweep] = None) -> Workload:
    """Two trackers of 3 x 2 modules and nothing else. Two-axis trackers stand in a
    north-south line (the southern one shades the other when the sun is low in the south),
    one-axis trackers (north-south axes) in an east-west line (they shade each other in the
    morning and evening)."""
    second = [0.0, gap_m, 2.5] if kind == 2 else [gap_m, 0.0, 2.5]
    gen = tracker_generator([[0.0, 0.0, 2.5], second], kind, n_u=3, n_v=2, modules_per_string=6)
    sw = sweep if sweep is not None else make_sweep(LAT_DEG, [20, 80, 172, 355], np.arange(5, 20), up_only=True)
    return Workload(f"tracker_pair_k{kind}", Scene(np.zeros((0, 3)), np.zeros((0, 3), np.int32)), gen, sw,
                    map_n, k, f"2 trackers (kind {kind}), {gap_m} m apart")


def c6_tracker_plant(seed: int = 6, sweep: Optional[Sweep] = None, map_n: int = 4096, k: int = 8,
                     n_x: int = 6, n_y: int = 3) -> Workload:
    """Two-axis tracker plant on uneven ground (the paper's Sec. 3.4 case): 18 trackers of
    7 x 4 modules (504 modules, 30,240 cells) on rolling terrain, one lattice pylon in the field."""
    rng = np.random.default_rng(seed)
    sx, sy = 22.0, 28.0
    xs = (np.arange(n_x) - (n_x - 1) / 2) * sx
    ys = (np.arange(n_y) - (n_y - 1) / 2) * sy
    X, Y = np.meshgrid(xs, ys, indexing="xy")
    x, y = X.ravel(), Y.ravel()
    half = max(abs(xs).max(), abs(ys).max()) + 120.0
    tv, tt, z_at = terrain(-half, -half, half, half, 64, rng)
    piv = np.stack([x, y, z_at(x, y) + 3.5], 1)
    gen = tracker_generator(piv, 2)
    m = _Mesh()
    m.add(tv, tt)
    px, py = xs[2] + sx / 2, ys[1] + sy / 2            # between trackers
    pv, pt = pylons(px, py, rng.uniform(0, 2 * np.pi, 1))
    pv = pv.copy()
    pv[..., 2] += float(z_at(px, py))
    m.add(pv, pt)
    sw = sweep if sweep is not None else year_sweep()
    return Workload("c6_tracker_plant", m.scene(), gen, sw, map_n, k,
                    f"{n_x * n_y} two-axis trackers of 7x4 modules on terrain, 1 pylon, N={map_n}, k={k}")


def c2_tracker_rows(seed: int = 2, n_pylons: int = 50, sweep: Optional[Sweep] = None, rows: int = 20,
                    map_n: int = 4096, k: int = 8) -> Workload:
    """The row plant on one-axis trackers: 20 north-south rows of 2 x 10 modules (400 modules,
    24,000 cells) turning about their axes, 4.5 m apart, ground plane, 50 lattice pylons."""
    rng = np.random.default_rng(seed)
    xs = (np.arange(rows) - (rows - 1) / 2) * 4.5
    piv = np.stack([xs, np.zeros(rows), np.full(rows, 2.0)], 1)
    gen = tracker_generator(piv, 1, n_u=2, n_v=10, modules_per_string=20)
    lo = np.array([xs.min() - 3.0, -10.0, 0.0])
    hi = np.array([xs.max() + 3.0, 10.0, 4.0])
    m = _Mesh()
    m.add(*ground_plane(lo[0] - 200, lo[1] - 200, hi[0] + 200, hi[1] + 200, 0.0))
    px, py = [], []
    while len(px) < n_pylons:
        x = rng.uniform(lo[0] - 60, hi[0] + 60)
        y = rng.uniform(lo[1] - 60, hi[1] + 60)
        if lo[0] - 5 <= x <= hi[0] + 5 and lo[1] - 5 <= y <= hi[1] + 5:
            continue
        px.append(x); py.append(y)
    m.add(*pylons(np.array(px), np.array(py), rng.uniform(0, 2 * np.pi, n_pylons)))
    sw = sweep if sweep is not None else year_sweep()
    return Workload("c2_tracker_rows", m.scene(), gen, sw, map_n, k,
                    f"{rows} one-axis tracker rows of 2x10 modules, {n_pylons} pylons, ground, N={map_n}, k={k}")


# --------------------------------------------------------------------------
# many generators in one scene
# --------------------------------------------------------------------------
def c7_stadium(seed: int = 7, sweep: Optional[Sweep] = None, n_gen: int = 88, n_u: int = 4, n_v: int = 14,
               map_n: int = 4096, k: int = 8, ring=(110.0, 90.0), slope_deg: float = 12.0) -> List[Workload]:
    """A stadium roof with many generators (the paper's Sec. 3.3 case: 88 generators of 14 x 4
    panels, each with its own orientation), here 4 panels along the ring and 14 down the roof.
    The generators sit around an elliptical ring on a roof that slopes toward the pitch; an
    outer wall ends just below them and four light towers stand inside the ring. Every
    generator's modules are part of the shared scene, so each generator is shaded by the
    others; each is evaluated with its own window and picture (one job per generator, all
    sharing the scene) and does not add itself again as occluders."""
    rng = np.random.default_rng(seed)
    a_r, b_r = ring
    beta = math.radians(slope_deg)
    w = n_u * MOD_W + (n_u - 1) * 0.02
    gens = []
    m = _Mesh()
    for i in range(n_gen):
        phi = 2.0 * math.pi * (i + 0.5) / n_gen
        c = np.array([a_r * math.cos(phi), b_r * math.sin(phi), 30.0])
        er = np.array([math.cos(phi) / a_r, math.sin(phi) / b_r, 0.0])      # outward normal of the ellipse
        er /= np.linalg.norm(er)
        et = np.array([-er[1], er[0], 0.0])                                # tangential, er x et = z
        up = math.cos(beta) * er + math.sin(beta) * np.array([0.0, 0.0, 1.0])   # rises outward
        U, V = MOD_W * et, MOD_L * up
        if np.cross(U, V)[2] < 0.0:
            U = -U
        uh, vh = U / MOD_W, V / MOD_L
        q = np.arange(n_u * n_v)
        iu, jv = q % n_u, q // n_u
        O = (c - 0.5 * w * uh)[None] + (iu * (MOD_W + 0.02))[:, None] * uh[None] + (jv * (MOD_L + 0.02))[:, None] * vh[None]
        g = Generator(np.ascontiguousarray(O), np.tile(U, (O.shape[0], 1)), np.tile(V, (O.shape[0], 1)), N_CU, N_CV,
                      portrait_substrings(), 3, (q // 14).astype(np.int32), add_as_occluders=False)
        gens.append(g)
        c0, c1, c2 = O, O + U, (O + U) + V
        m.add(np.stack([c0, c1, c2], 1), np.array([[0, 1, 2]]))
        m.add(np.stack([c0, c2, O + V], 1), np.array([[0, 1, 2]]))
    # outer wall: 176 segments ending just below the panels; four light towers
    n_w = 2 * n_gen
    ph = 2.0 * math.pi * (np.arange(n_w) + 0.5) / n_w
    grow = 1.0 + (n_v * MOD_L * math.cos(beta) + 1.0) / min(a_r, b_r)
    wx, wy = a_r * grow * np.cos(ph), b_r * grow * np.sin(ph)
    seg = 2.0 * math.pi * max(a_r, b_r) * grow / n_w * 1.05
    yaw = np.arctan2(b_r * np.cos(ph), -a_r * np.sin(ph))
    top = 29.5
    m.add(*boxes(wx, wy, seg, 1.0, 0.0, top, yaw, floor=False))
    tw = rng.uniform(0.0, 2.0 * math.pi) + np.arange(4) * math.pi / 2
    m.add(*boxes(0.7 * a_r * np.cos(tw), 0.7 * b_r * np.sin(tw), 2.0, 2.0, 0.0, 55.0, 0.0, floor=False))
    scene = m.scene()
    sw = sweep if sweep is not None else year_sweep()
    return [Workload(f"c7_stadium_g{i}", scene, g, sw, map_n, k,
                     f"generator {i} of {n_gen} ({n_u}x{n_v} modules) on a stadium ring, N={map_n}, k={k}")
            for i, g in enumerate(gens)]


def c7_stadium_small(sweep: Optional[Sweep] = None) -> List[Workload]:
    """Ten generators of 2 x 4 modules on a 30 m x 24 m ring, N = 256, k = 2, every 37th sun of
    the year: a stadium small enough for the oracle in seconds that still shades itself."""
    if sweep is None:
        yr = year_sweep()
        sweep = yr.subset(np.arange(0, yr.n, 37))
    return c7_stadium(sweep=sweep, n_gen=10, n_u=2, n_v=4, map_n=256, k=2, ring=(30.0, 24.0))


def sky_directions(n: int) -> np.ndarray:
    """n directions over the sky hemisphere, each standing for an equal solid angle: a golden-angle
    spiral with heights z_j = (j + 1/2) / n (equal bands of height hold equal solid angle)."""
    j = np.arange(n, dtype=np.float64)
    z = (j + 0.5) / n
    phi = j * math.pi * (3.0 - math.sqrt(5.0))
    r = np.sqrt(1.0 - z * z)
    return np.stack([r * np.cos(phi), r * np.sin(phi), z], 1)


# --------------------------------------------------------------------------
# the configurations
# --------------------------------------------------------------------------
def c1_tiny(d_poa: float = 0.0) -> Workload:
    """One 60-cell module, 30 deg south, one 0.2 x 0.2 x 4 m pole 3 m south; day 355, 24 hours."""
    b = math.radians(30.0)
    gen = Generator(np.array([[-MOD_W / 2, 0.0, 0.0]]), np.array([[MOD_W, 0.0, 0.0]]),
                    np.array([[0.0, MOD_L * math.cos(b), MOD_L * math.sin(b)]]),
                    N_CU, N_CV, portrait_substrings(), 3, np.zeros(1, np.int32))
    m = _Mesh()
    m.add(*boxes(0.0, -3.0, 0.2, 0.2, 0.0, 4.0, 0.0, floor=True))
    sw = make_sweep(LAT_DEG, [355], np.arange(24), dni=1000.0, d_poa=d_poa)
    return Workload("c1_tiny_pole", m.scene(), gen, sw, 1024, 16,
                    "1 module, 12-triangle pole, day 355 hourly, N=1024, k=16")


def c2_row_plant(seed: int = 2, n_pylons: int = 50, sweep: Optional[Sweep] = None,
                 rows: int = 20, per_row: int = 20, map_n: int = 4096, k: int = 8,
                 gap: float = 0.02) -> Workload:
    """20 x 20 fixed-tilt rows at 3.9 m pitch, ground plane, 50 lattice pylons, full year."""
    rng = np.random.default_rng(seed)
    gen = module_rows(rows, per_row, gap=gap)
    lo, hi = gen_bbox(gen)
    m = _Mesh()
    m.add(*ground_plane(lo[0] - 200, lo[1] - 200, hi[0] + 200, hi[1] + 200, 0.0))
    px, py = [], []
    while len(px) < n_pylons:
        x = rng.uniform(lo[0] - 60, hi[0] + 60)
        y = rng.uniform(lo[1] - 60, hi[1] + 60)
        if lo[0] - 5 <= x <= hi[0] + 5 and lo[1] - 5 <= y <= hi[1] + 5:
            continue
        px.append(x); py.append(y)
    if n_pylons:
        m.add(*pylons(np.array(px), np.array(py), rng.uniform(0, 2 * np.pi, n_pylons)))
    sw = sweep if sweep is not None else year_sweep()
    return Workload("c2_row_plant", m.scene(), gen, sw, map_n, k,
                    f"{rows}x{per_row} modules, {n_pylons} pylons, ground, N={map_n}, k={k}")


def c3_rooftop(seed: int = 3, sweep: Optional[Sweep] = None, n_buildings: int = 200,
               n_trees: int = 1000, map_n: int = 8192, k: int = 8) -> Workload:
    """2,000 flat landscape modules on a 64 x 48 m roof, 200 buildings, 1,000 trees."""
    rng = np.random.default_rng(seed)
    nx, ny = 40, 50
    m_idx = np.arange(nx * ny)
    ix, iy = m_idx % nx, m_idx // nx
    x0, y0 = -nx * MOD_L / 2, ny * MOD_W / 2
    O = np.stack([x0 + ix * MOD_L, y0 - iy * MOD_W, np.full(nx * ny, 10.05)], 1)
    U = np.tile([0.0, -MOD_W, 0.0], (nx * ny, 1))      # 6-cell side, pointing south
    V = np.tile([MOD_L, 0.0, 0.0], (nx * ny, 1))       # 10-cell side, pointing east; U x V = +z
    gen = Generator(np.ascontiguousarray(O), U, V, N_CU, N_CV, portrait_substrings(), 3,
                    (m_idx // 20).astype(np.int32))
    m = _Mesh()
    m.add(*boxes(0.0, 0.0, 64.0, 48.0, 0.0, 10.0, 0.0, floor=False))
    hx, hy = 32.0 + 5.0, 24.0 + 5.0
    bx, by, bs = [], [], []
    while len(bx) < n_buildings:
        x, y = _annulus(rng, 1, 60.0, 400.0)
        sx, sy = rng.uniform(10, 30, 2)
        rad = 0.5 * math.hypot(sx, sy)
        if abs(x[0]) < hx + rad and abs(y[0]) < hy + rad:
            continue
        bx.append(x[0]); by.append(y[0]); bs.append((sx, sy))
    if n_buildings:
        bs = np.array(bs)
        h = rng.lognormal(math.log(15.0), 0.5, n_buildings)
        m.add(*boxes(np.array(bx), np.array(by), bs[:, 0], bs[:, 1], 0.0, h,
                     rng.uniform(0, 2 * np.pi, n_buildings), floor=False))
    if n_trees:
        tx, ty = _annulus(rng, n_trees, 40.0, 300.0)
        m.add(*trees(tx, ty, rng.uniform(1.0, 4.0, n_trees)))
    sw = sweep if sweep is not None else year_sweep()
    return Workload("c3_rooftop_bipv", m.scene(), gen, sw, map_n, k,
                    f"2000 modules on a roof, {n_buildings} buildings, {n_trees} trees, N={map_n}, k={k}")


def map_size_rule(gen: Generator, k: int = 8) -> int:
    """Power of two at least twice the generator extent in sample spacings, in [2048, 8192]."""
    lo, hi = gen_bbox(gen)
    ext = float(max(hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]))
    need = 2.0 * ext / (CELL / k)
    n = 1 << max(0, int(math.ceil(math.log2(max(need, 1.0)))))
    return int(min(max(n, 2048), 8192))


def site_scene(rng: np.random.Generator, n_tri_target: float, r0: float = 50.0, r1: float = 300.0,
               ground: bool = True) -> Scene:
    """Trees / pylons / buildings (70 / 20 / 10 % of the triangle budget) in an annulus."""
    m = _Mesh()
    if ground:
        m.add(*ground_plane(-r1, -r1, r1, r1, 0.0))
    n_t = int(round(0.7 * n_tri_target / 516))
    n_p = int(round(0.2 * n_tri_target / 2016))
    n_b = int(round(0.1 * n_tri_target / 10))
    if n_t:
        x, y = _annulus(rng, n_t, r0, r1)
        m.add(*trees(x, y, rng.uniform(1.0, 4.0, n_t)))
    if n_p:
        x, y = _annulus(rng, n_p, r0, r1)
        m.add(*pylons(x, y, rng.uniform(0, 2 * np.pi, n_p)))
    if n_b:
        x, y = _annulus(rng, n_b, r0 + 10, r1)
        m.add(*boxes(x, y, rng.uniform(10, 30, n_b), rng.uniform(10, 30, n_b), 0.0,
                     rng.lognormal(math.log(15.0), 0.5, n_b), rng.uniform(0, 2 * np.pi, n_b),
                     floor=False))
    return m.scene()


def site_generator(n_cells: int) -> Generator:
    n_mod = max(1, int(round(n_cells / (N_CU * N_CV))))
    per_row = min(20, n_mod)
    n_rows = (n_mod + per_row - 1) // per_row
    g = module_rows(n_rows, per_row, n_mod=n_mod, x0=-per_row * (MOD_W + 0.02) / 2,
                    y0=-n_rows * 3.9 / 2)
    return g


def _loguniform(rng, lo, hi, size=None):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size))


def c4_batched(seed: int = 4, n_sites: int = 64, sweep: Optional[Sweep] = None,
               tri_range=(1e3, 2e6), cell_range=(60, 24000), k: int = 8) -> List[Workload]:
    """64 sites of uneven size, each with a full-year sweep, for one persistent launch."""
    rng = np.random.default_rng(seed)
    sw = sweep if sweep is not None else year_sweep()
    out = []
    for i in range(n_sites):
        nt = float(_loguniform(rng, *tri_range))
        nc = int(round(float(_loguniform(rng, *cell_range))))
        sc = site_scene(rng, nt)
        g = site_generator(nc)
        out.append(Workload(f"c4_site{i:02d}", sc, g, sw, map_size_rule(g, k), k,
                            f"site {i}: {sc.n_tri} tris, {g.n_cells} cells"))
    return out


@dataclasses.dataclass
class Request:
    arrival_s: float
    scene_id: int
    sun_idx: np.ndarray
    n_cells: int
    map_n: int


def serving_stream(seed: int = 5, rate_hz: float = 200.0, duration_s: float = 60.0,
                   n_scenes: int = 256, zipf_s: float = 1.1, sun_max: int = 4381,
                   cell_range=(60, 24000), year: Optional[Sweep] = None, k: int = 8):
    """Poisson arrivals of shading jobs over a Zipf-popular scene pool (request list only)."""
    rng = np.random.default_rng(seed)
    yr = year if year is not None else year_sweep()
    w = 1.0 / np.arange(1, n_scenes + 1) ** zipf_s
    w /= w.sum()
    t = 0.0
    reqs = []
    while True:
        t += rng.exponential(1.0 / rate_hz)
        if t >= duration_s:
            break
        sid = int(rng.choice(n_scenes, p=w))
        ns = int(min(yr.n, max(1, round(float(_loguniform(rng, 1, min(sun_max, yr.n)))))))
        start = int(rng.integers(0, yr.n))
        idx = (start + np.arange(ns)) % yr.n
        nc = int(round(float(_loguniform(rng, *cell_range))))
        g = site_generator(nc)
        reqs.append(Request(t, sid, idx.astype(np.int64), g.n_cells, map_size_rule(g, k)))
    return reqs


def serving_scene(seed: int, scene_id: int, tri_range=(1e4, 1e6)) -> Scene:
    rng = np.random.default_rng([seed, scene_id])
    return site_scene(rng, float(_loguniform(rng, *tri_range)))


# --------------------------------------------------------------------------
# tiny random cases for parity and pin tests
# --------------------------------------------------------------------------
def random_tiny(seed: int, n_boxes: int = 6, n_loose: int = 20, n_mod_side: int = 2,
                tilt_deg: float = 25.0, map_n: int = 200, k: int = 3, n_sun: int = 6,
                d_poa: float = 50.0) -> Workload:
    """A small module grid with boxes around it and loose triangles floating above it.

    Occluders never intersect a module: boxes stand outside the generator's
    footprint (plus 0.5 m), loose triangles lie above its highest corner
    (plus 0.5 m), so every exact occlusion has a definite side.
    """
    rng = np.random.default_rng(seed)
    gen = module_rows(n_mod_side, n_mod_side, tilt_deg=tilt_deg, pitch=2.6, z0=0.3,
                      modules_per_string=max(1, n_mod_side))
    lo, hi = gen_bbox(gen)
    ctr = 0.5 * (lo + hi)
    m = _Mesh()
    bx, by, bsx, bsy = [], [], [], []
    while len(bx) < n_boxes:
        x, y = ctr[0] + rng.uniform(-9, 9), ctr[1] + rng.uniform(-9, 9)
        sx, sy = rng.uniform(0.1, 1.5, 2)
        r = 0.5 * math.hypot(sx, sy)
        if lo[0] - 0.5 - r < x < hi[0] + 0.5 + r and lo[1] - 0.5 - r < y < hi[1] + 0.5 + r:
            continue
        bx.append(x); by.append(y); bsx.append(sx); bsy.append(sy)
    if n_boxes:
        m.add(*boxes(np.array(bx), np.array(by), np.array(bsx), np.array(bsy),
                     rng.uniform(-0.5, 0.2, n_boxes), rng.uniform(1.0, 5.0, n_boxes),
                     rng.uniform(0, 2 * np.pi, n_boxes)))
    if n_loose:
        c = np.stack([ctr[0] + rng.uniform(-7, 7, n_loose), ctr[1] + rng.uniform(-7, 7, n_loose),
                      hi[2] + 1.3 + rng.uniform(0.0, 3.0, n_loose)], 1)[:, None, :]
        v = c + rng.uniform(-0.8, 0.8, (n_loose, 3, 3))
        m.add(v, np.array([[0, 1, 2]]))
    days = rng.integers(1, 366, n_sun)
    hours = rng.integers(7, 18, n_sun).astype(np.float64)
    s = cooper_sun(LAT_DEG, days, hours)
    sw = Sweep(np.ascontiguousarray(s), np.full(n_sun, 900.0), np.full(n_sun, d_poa),
               np.full(n_sun, 1.0), days.astype(np.int32), hours)
    return Workload(f"tiny{seed}", m.scene(), gen, sw, map_n, k, "random tiny case")
