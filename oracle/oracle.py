"""ctypes loader for the C oracle in ``pv3d_oracle.c``.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark use it; the product path never imports it. It shares no
code with the HIP library.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pv3d_oracle.c")
LIB = os.path.join(HERE, "liboracle_pv3d.so")
DMAX = (1 << 24) - 1

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: binary64, no contraction, OpenMP over suns."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC",
           "-shared", "-Wall", "-Wextra", "-o", tmp, SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


def _bind(path: str):
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i64, i32, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    L.oracle_evaluate.restype = i64
    L.oracle_evaluate.argtypes = [P, i64, P, i64, P, P, P, i64, i32, i32, P, i32, P, i32,
                                  P, P, P, P, i64, i32, i32, P, P, P, P, P, P, i32, P, P]
    L.oracle_sky_view.restype = i64
    L.oracle_sky_view.argtypes = [P, i64, P, i64, P, P, P, i64, i32, i32, P, i32, P, i32, P, i64, i32, i32, P, i32]
    L.oracle_view.restype = None
    L.oracle_view.argtypes = [P, i64, P, P, P, i64, P, f64, i32, P, P, P]
    L.oracle_raster.restype = None
    L.oracle_raster.argtypes = [P, i64, i32, P, P]
    L.oracle_string_power.restype = f64
    L.oracle_string_power.argtypes = [P, i64]
    L.oracle_evaluate_tracked.restype = i64
    L.oracle_evaluate_tracked.argtypes = [P, i64, P, i64, P, P, P, i64, i32, i32, P, i32, P, i32, P, i32, P,
                                          P, P, P, P, i64, i32, i32, P, P, P, P, P, P, i32, P, P]
    L.oracle_pose.restype = None
    L.oracle_pose.argtypes = [P, i32, P, P, P, P, i64, P, P, P, P]
    L.oracle_cell_voltage.restype = f64
    L.oracle_cell_voltage.argtypes = [P, f64, f64]
    L.oracle_string_voltage.restype = f64
    L.oracle_string_voltage.argtypes = [P, P, P, i64, f64]
    L.oracle_string_mpp.restype = f64
    L.oracle_string_mpp.argtypes = [P, P, P, i64]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        _lib = _bind(LIB)
    return _lib


class use_library:
    """Temporarily route this module's calls to another build of the oracle source
    (the mutation tests use it to check that the pins catch planted mistakes)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        self.saved = lib()
        _lib = _bind(self.path)
        return self

    def __exit__(self, *exc):
        global _lib
        _lib = self.saved
        return False


def build_variant(source_text: str, out_path: str) -> str:
    """Compile a modified copy of the oracle source (same flags) to out_path."""
    src = out_path[:-3] + ".c"
    with open(src, "w") as f:
        f.write(source_text)
    subprocess.run(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                    "-fPIC", "-shared", "-w", "-o", out_path, src, "-lm"], check=True)
    return out_path


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class OracleResult:
    def __init__(self, counts, power, power_ref, energy, maps, bits, outside):
        self.counts = counts
        self.power = power
        self.power_ref = power_ref
        self.energy = energy
        self.maps = maps
        self.bits = bits
        self.outside = outside

    @property
    def loss(self) -> float:
        return 1.0 - self.energy[0] / self.energy[1] if self.energy[1] > 0 else 0.0


def evaluate(scene, gen, sweep, map_n: int, k: int, export_maps: bool = False,
             export_bits: bool = False, threads: int = 0) -> OracleResult:
    """Run the oracle over a whole sweep (inputs from ``workloads``)."""
    L = lib()
    xyz = _c(scene.xyz, np.float64).reshape(-1, 3)
    tri = _c(scene.tri, np.int32).reshape(-1, 3)
    org, eu, ev = (_c(a, np.float64) for a in (gen.origin, gen.edge_u, gen.edge_v))
    cs = _c(gen.cell_substring, np.int32)
    ms = _c(gen.module_string, np.int32)
    s = _c(sweep.sun_xyz, np.float64)
    dni, dp, dt = (_c(a, np.float64) for a in (sweep.dni, sweep.d_poa, sweep.dt_h))
    ns = sweep.n
    cells = gen.n_cells
    counts = np.zeros((ns, cells), np.uint32)
    pw = np.zeros(ns)
    pr = np.zeros(ns)
    en = np.zeros(2)
    maps = np.zeros((ns, map_n, map_n), np.uint32) if export_maps else None
    words = (k * k + 31) // 32
    bits = np.zeros((ns, cells, words), np.uint32) if export_bits else None
    dio = _diode(getattr(gen, "diode", None))
    svf = getattr(gen, "sky_view", None)
    if svf is not None:
        svf = _c(svf, np.float64).reshape(-1)
        assert svf.shape[0] == gen.n_cells
    if getattr(gen, "trackers", None) is not None:
        trk = _c(gen.trackers, np.float64).reshape(-1, 7)
        mt = _c(gen.module_tracker, np.int32)
        out = L.oracle_evaluate_tracked(_p(xyz), xyz.shape[0], _p(tri), tri.shape[0], _p(org), _p(eu), _p(ev),
                                        gen.n_mod, gen.n_cu, gen.n_cv, _p(cs), gen.n_sub, _p(ms),
                                        1 if gen.add_as_occluders else 0, _p(trk), trk.shape[0], _p(mt),
                                        _p(s), _p(dni), _p(dp), _p(dt), ns, map_n, k, _p(counts), _p(pw), _p(pr),
                                        _p(en), _p(maps), _p(bits), threads, _p(dio), _p(svf))
    else:
        out = L.oracle_evaluate(_p(xyz), xyz.shape[0], _p(tri), tri.shape[0], _p(org), _p(eu), _p(ev),
                                gen.n_mod, gen.n_cu, gen.n_cv, _p(cs), gen.n_sub, _p(ms),
                                1 if gen.add_as_occluders else 0, _p(s), _p(dni), _p(dp), _p(dt), ns,
                                map_n, k, _p(counts), _p(pw), _p(pr), _p(en), _p(maps), _p(bits), threads,
                                _p(dio), _p(svf))
    if out < 0:
        raise ValueError("oracle rejected its arguments")
    return OracleResult(counts, pw, pr, en, maps, bits, int(out))


def sky_view(scene, gen, dirs, map_n: int, k: int, threads: int = 0) -> np.ndarray:
    """Per-cell sky view factors [n_cells] of a fixed generator over sky directions dirs [n, 3]."""
    L = lib()
    xyz = _c(scene.xyz, np.float64).reshape(-1, 3)
    tri = _c(scene.tri, np.int32).reshape(-1, 3)
    org, eu, ev = (_c(a, np.float64) for a in (gen.origin, gen.edge_u, gen.edge_v))
    cs = _c(gen.cell_substring, np.int32)
    ms = _c(gen.module_string, np.int32)
    d = _c(dirs, np.float64).reshape(-1, 3)
    out = np.zeros(gen.n_cells)
    r = L.oracle_sky_view(_p(xyz), xyz.shape[0], _p(tri), tri.shape[0], _p(org), _p(eu), _p(ev), gen.n_mod,
                          gen.n_cu, gen.n_cv, _p(cs), gen.n_sub, _p(ms), 1 if gen.add_as_occluders else 0, _p(d),
                          d.shape[0], map_n, k, _p(out), threads)
    if r != 0:
        raise ValueError(f"oracle sky view: {r}")
    return out


def _diode(d) -> Optional[np.ndarray]:
    """Single-diode parameters as the C side takes them: Isc_ref, G_ref, I0, a, Rs, Rsh, Vb."""
    if d is None:
        return None
    a = _c(d, np.float64).reshape(-1)
    if a.shape[0] != 7:
        raise ValueError("diode parameters: Isc_ref, G_ref, I0, a, Rs, Rsh, Vb")
    return a


def cell_voltage(d, G: float, I: float) -> float:
    """Voltage of one cell of the single-diode model at irradiance G and current I."""
    dd = _diode(d)
    return float(lib().oracle_cell_voltage(_p(dd), float(G), float(I)))


def string_voltage(d, g, sub_len, I: float) -> float:
    """Voltage of a string (cell irradiances g, substring after substring, sub_len cells each)."""
    dd, gg, sl = _diode(d), _c(g, np.float64), _c(sub_len, np.int32)
    assert int(sl.sum()) == gg.shape[0]
    return float(lib().oracle_string_voltage(_p(dd), _p(gg), _p(sl), sl.shape[0], float(I)))


def string_mpp(d, g, sub_len) -> float:
    """Maximum power of such a string under the single-diode model."""
    dd, gg, sl = _diode(d), _c(g, np.float64), _c(sub_len, np.int32)
    assert int(sl.sum()) == gg.shape[0]
    return float(lib().oracle_string_mpp(_p(dd), _p(gg), _p(sl), sl.shape[0]))


def view(scene, gen, sun, map_n: int, dni: float = 1000.0):
    """Light-space view and per-module beam / bias of one sun (for brute-force pins)."""
    L = lib()
    xyz = _c(scene.xyz, np.float64).reshape(-1, 3)
    org, eu, ev = (_c(a, np.float64) for a in (gen.origin, gen.edge_u, gen.edge_v))
    s = _c(sun, np.float64)
    w = np.zeros(17)
    beam = np.zeros(gen.n_mod)
    bias = np.zeros(gen.n_mod, np.int32)
    L.oracle_view(_p(xyz), xyz.shape[0], _p(org), _p(eu), _p(ev), gen.n_mod, _p(s), dni, map_n,
                  _p(w), _p(beam), _p(bias))
    return dict(e1=w[0:3], e2=w[3:6], d=w[6:9], ox=w[9], oy=w[10], itx=w[11], ity=w[12],
                znear=w[13], izd=w[14], valid=bool(w[15]), n=int(w[16]), beam=beam, bias=bias)


def pose(gen, sun):
    """The generator's modules posed for one sun: (origin, edge_u, edge_v), each [M, 3]."""
    L = lib()
    org, eu, ev = (_c(a, np.float64) for a in (gen.origin, gen.edge_u, gen.edge_v))
    trk = _c(gen.trackers, np.float64).reshape(-1, 7)
    mt = _c(gen.module_tracker, np.int32)
    s = _c(sun, np.float64)
    o2, u2, v2 = (np.zeros_like(org) for _ in range(3))
    L.oracle_pose(_p(trk), trk.shape[0], _p(mt), _p(org), _p(eu), _p(ev), gen.n_mod, _p(s), _p(o2), _p(u2), _p(v2))
    return o2, u2, v2


def raster(tris_light: np.ndarray, map_n: int, with_cover: bool = True):
    """Raster light-space triangles [n,3,3]; returns (map, cover)."""
    L = lib()
    t = _c(tris_light, np.float64).reshape(-1, 3, 3)
    m = np.zeros((map_n, map_n), np.uint32)
    c = np.zeros((map_n, map_n), np.uint32) if with_cover else None
    L.oracle_raster(_p(t), t.shape[0], map_n, _p(m), _p(c))
    return m, c


def string_power(caps) -> float:
    c = _c(caps, np.float64)
    return float(lib().oracle_string_power(_p(c), c.shape[0]))
