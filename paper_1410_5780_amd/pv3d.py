"""ctypes binding of libpv3d (include/pv3d.h): argument marshalling only.

Every step of the shading path runs in the library's HIP kernels; this module
converts numpy arrays and torch device tensors to pointers, checks status
codes, and shapes the results. It raises if the shared library is missing:
there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpv3d.so")

OK, EINVAL, ENOMEM, ENOENT, EDEVICE, ERANGE, EBUSY, ECANCELED = 0, -1, -2, -3, -4, -5, -6, -7
TUNE_LOAD, TUNE_SAVE, TUNE_CLEAR = 0, 1, 2
EXPORT_DEPTH, EXPORT_BITS, SEPARATE_TEST, FULL_RASTER = 1, 2, 4, 8
BATCH_ANY_XCD = 1
STAGES = ("tri_setup", "bin_scan", "bin_scatter", "raster", "sample_test", "setup", "loss")
STAGE = {n: i for i, n in enumerate(STAGES)}
N_STAGES = len(STAGES)
DEPTH_MAX = (1 << 24) - 1

_P = ctypes.c_void_p
_i32, _i64, _u32, _u64, _f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double


class Module(ctypes.Structure):
    _fields_ = [("origin", _f64 * 3), ("edge_u", _f64 * 3), ("edge_v", _f64 * 3), ("n_cu", _i32), ("n_cv", _i32)]


class Tracker(ctypes.Structure):
    _fields_ = [("kind", _i32), ("reserved", _i32), ("pivot", _f64 * 3), ("axis", _f64 * 3)]


class Diode(ctypes.Structure):
    _fields_ = [("isc_ref", _f64), ("g_ref", _f64), ("i0", _f64), ("a", _f64), ("rs", _f64), ("rsh", _f64),
                ("v_bypass", _f64)]


class Params(ctypes.Structure):
    _fields_ = [("map_n", _i32), ("k", _i32), ("flags", _u32), ("tile", _i32), ("bin_limit", _i32),
                ("reserved", _i32)]


class Outputs(ctypes.Structure):
    _fields_ = [("cell_counts", _P), ("power", _P), ("power_ref", _P), ("energy", _P),
                ("depth_maps", _P), ("shaded_bits", _P), ("on_device", _i32)]


class Job(ctypes.Structure):
    _fields_ = [("scene", _u64), ("gen", _u64), ("sun_xyz", _P), ("dni", _P), ("d_poa", _P), ("dt_h", _P),
                ("n_sun", _i64), ("params", Params), ("out", Outputs)]


class Pv3dError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"pv3d error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libpv3d.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              "or python paper_1410_5780_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        L.pv3d_create.argtypes = [_i32, _u64, ctypes.POINTER(_P)]
        L.pv3d_destroy.argtypes = [_P]
        L.pv3d_destroy.restype = None
        L.pv3d_last_error.argtypes = [_P]
        L.pv3d_last_error.restype = ctypes.c_char_p
        L.pv3d_scene_load.argtypes = [_P, _P, _i64, _P, _i64, ctypes.POINTER(_u64)]
        L.pv3d_scene_release.argtypes = [_P, _u64]
        L.pv3d_generator_define.argtypes = [_P, _P, _i64, _P, _i32, _P, _i32, ctypes.POINTER(_u64)]
        L.pv3d_generator_define_tracked.argtypes = [_P, _P, _i64, _P, _i32, _P, _i32, _P, _i32, _P,
                                                    ctypes.POINTER(_u64)]
        L.pv3d_generator_release.argtypes = [_P, _u64]
        L.pv3d_generator_set_diode.argtypes = [_P, _u64, ctypes.POINTER(Diode)]
        L.pv3d_generator_set_sky.argtypes = [_P, _u64, _P]
        L.pv3d_sky_view.argtypes = [_P, _u64, _u64, _P, _i64, ctypes.POINTER(Params), _P]
        L.pv3d_sun_cooper.argtypes = [_f64, _P, _P, _i64, _P]
        L.pv3d_evaluate.argtypes = [_P, _u64, _u64, _P, _P, _P, _P, _i64, ctypes.POINTER(Params),
                                    ctypes.POINTER(Outputs), _P]
        L.pv3d_path_stats.argtypes = [_P, ctypes.POINTER(_i64 * 4)]
        L.pv3d_evaluate_noalloc.argtypes = [_P, _u64, _u64, _P, _P, _P, _P, _i64, ctypes.POINTER(Params),
                                            ctypes.POINTER(Outputs), _P]
        L.pv3d_evaluate_batched.argtypes = [_P, ctypes.POINTER(Job), _i64, _P]
        L.pv3d_autotune.argtypes = [_P, ctypes.POINTER(Job), _i32, ctypes.POINTER(_f64)]
        L.pv3d_autotune_cache.argtypes = [_P, ctypes.c_char_p, _i32]
        L.pv3d_batch_stats.argtypes = [_P, ctypes.POINTER(_i64 * 7)]
        L.pv3d_batch_limits.argtypes = [_P, _i32, _i64, _u32]
        L.pv3d_serve_stats.argtypes = [_P, ctypes.POINTER(_i64 * 4)]
        L.pv3d_submit.argtypes = [_P, ctypes.POINTER(Job), ctypes.POINTER(_u64)]
        L.pv3d_poll.argtypes = [_P, _u64, ctypes.POINTER(_i32)]
        L.pv3d_wait.argtypes = [_P, _u64]
        L.pv3d_cancel.argtypes = [_P, _u64]
        L.pv3d_profile_enable.argtypes = [_P, _u32]
        L.pv3d_profile_read.argtypes = [_P, _i32, ctypes.POINTER(_f64), ctypes.POINTER(_i64)]
        L.pv3d_profile_sample.argtypes = [_P, _i32]
        L.pv3d_profile_busy.argtypes = [_P, _i32, ctypes.POINTER(_f64), ctypes.POINTER(_i64)]
        for f in ("pv3d_profile_enable", "pv3d_profile_read", "pv3d_profile_sample", "pv3d_profile_busy", "pv3d_create", "pv3d_scene_load", "pv3d_scene_release", "pv3d_generator_define",
                  "pv3d_generator_define_tracked", "pv3d_generator_release", "pv3d_generator_set_diode", "pv3d_generator_set_sky", "pv3d_sky_view",
                  "pv3d_sun_cooper", "pv3d_evaluate", "pv3d_evaluate_batched",
                  "pv3d_autotune", "pv3d_batch_stats", "pv3d_batch_limits", "pv3d_serve_stats",
                  "pv3d_submit", "pv3d_poll", "pv3d_wait", "pv3d_cancel"):
            getattr(L, f).restype = _i32
        _lib = L
    return _lib


_side: dict = {}


class _Ordered:
    """The stream an asynchronous call runs on, in the order of torch stream `st`. torch's
    default stream is the null stream (handle 0), which the C ABI would read as the context's
    own stream, not ordered with torch's work: such calls run on a side stream that first waits
    for `st`, and `st` waits for the side stream afterwards."""

    def __init__(self, st):
        import torch
        self.st, self.run = st, st
        if int(st.cuda_stream) == 0:
            dev = st.device
            if dev not in _side:
                _side[dev] = torch.cuda.Stream(device=dev)
            self.run = _side[dev]

    def __enter__(self) -> ctypes.c_void_p:
        if self.run is not self.st:
            self.run.wait_stream(self.st)
        return ctypes.c_void_p(int(self.run.cuda_stream))

    def __exit__(self, *exc):
        if self.run is not self.st:
            self.st.wait_stream(self.run)
        return False


def _ptr(a) -> Optional[int]:
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return int(a.data_ptr())            # torch tensor


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _check(code: int, ctx=None):
    if code != OK:
        raise Pv3dError(code, lib().pv3d_last_error(ctx).decode(errors="replace"))


def sun_cooper(lat_deg: float, day, hour) -> np.ndarray:
    day = _c(day, np.int32).ravel()
    hour = _c(hour, np.float64).ravel()
    out = np.zeros((day.shape[0], 3))
    _check(lib().pv3d_sun_cooper(lat_deg, _ptr(day), _ptr(hour), day.shape[0], _ptr(out)))
    return out


class Result:
    def __init__(self, counts, power, power_ref, energy, maps=None, bits=None):
        self.counts, self.power, self.power_ref, self.energy = counts, power, power_ref, energy
        self.maps, self.bits = maps, bits

    @property
    def loss(self) -> float:
        e = np.asarray(self.energy if isinstance(self.energy, np.ndarray) else self.energy.cpu().numpy())
        return float(1.0 - e[0] / e[1]) if e[1] > 0 else 0.0


def modules_of(gen) -> ctypes.Array:
    arr = (Module * gen.n_mod)()
    for m in range(gen.n_mod):
        arr[m].origin[:] = [float(x) for x in gen.origin[m]]
        arr[m].edge_u[:] = [float(x) for x in gen.edge_u[m]]
        arr[m].edge_v[:] = [float(x) for x in gen.edge_v[m]]
        arr[m].n_cu, arr[m].n_cv = int(gen.n_cu), int(gen.n_cv)
    return arr


def _torch_first():
    """Device arrays cross the ABI as torch tensors. torch carries a HIP runtime of its own, and
    when the library's runtime starts first torch no longer finds the GPU, so start torch's first
    whenever torch is importable."""
    try:
        import torch
    except ImportError:
        return
    try:
        if torch.cuda.is_available():
            torch.cuda.init()
    except Exception:
        pass


class Context:
    """One library context on one device (owns a HIP stream and an HBM budget)."""

    def __init__(self, device: int = 0, budget_bytes: int = 0):
        _torch_first()
        h = _P()
        _check(lib().pv3d_create(device, budget_bytes, ctypes.byref(h)))
        self.h = h
        self._keep = []

    def close(self):
        if self.h:
            lib().pv3d_destroy(self.h)
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def profile_enable(self, stage_mask: int):
        _check(lib().pv3d_profile_enable(self.h, stage_mask), self.h)

    def profile_sample(self, every: int):
        """Time only every n-th launch of each profiled stage."""
        _check(lib().pv3d_profile_sample(self.h, int(every)), self.h)

    def profile_read(self, stage: int):
        """(summed milliseconds, launches) of one stage since profiling was enabled."""
        ms, n = _f64(), _i64()
        _check(lib().pv3d_profile_read(self.h, stage, ctypes.byref(ms), ctypes.byref(n)), self.h)
        return ms.value, n.value

    def profile_busy(self, stage: int):
        """(milliseconds during which at least one timed launch of the stage ran, suns covered)."""
        ms, n = _f64(), _i64()
        _check(lib().pv3d_profile_busy(self.h, stage, ctypes.byref(ms), ctypes.byref(n)), self.h)
        return ms.value, n.value

    def load_scene(self, scene) -> int:
        xyz = _c(scene.xyz, np.float64).reshape(-1, 3)
        tri = _c(scene.tri, np.int32).reshape(-1, 3)
        h = _u64()
        _check(lib().pv3d_scene_load(self.h, _ptr(xyz), xyz.shape[0], _ptr(tri), tri.shape[0], ctypes.byref(h)), self.h)
        return h.value

    def release_scene(self, h: int):
        _check(lib().pv3d_scene_release(self.h, h), self.h)

    def define_generator(self, gen) -> int:
        mods = modules_of(gen)
        cs = _c(gen.cell_substring, np.int32)
        ms = _c(gen.module_string, np.int32)
        h = _u64()
        occ = 1 if gen.add_as_occluders else 0
        trk = getattr(gen, "trackers", None)
        if trk is None:
            _check(lib().pv3d_generator_define(self.h, ctypes.addressof(mods), gen.n_mod, _ptr(cs), int(gen.n_sub),
                                               _ptr(ms), occ, ctypes.byref(h)), self.h)
            return self._with_diode(h.value, gen)
        t = np.asarray(trk, np.float64).reshape(-1, 7)
        arr = (Tracker * t.shape[0])()
        for i, row in enumerate(t):
            arr[i].kind = int(row[0])
            arr[i].reserved = 0
            arr[i].pivot[:] = [float(x) for x in row[1:4]]
            arr[i].axis[:] = [float(x) for x in row[4:7]]
        mt = _c(gen.module_tracker, np.int32)
        _check(lib().pv3d_generator_define_tracked(self.h, ctypes.addressof(mods), gen.n_mod, _ptr(cs),
                                                   int(gen.n_sub), _ptr(ms), occ, ctypes.addressof(arr), t.shape[0],
                                                   _ptr(mt), ctypes.byref(h)), self.h)
        return self._with_diode(h.value, gen)

    def _with_diode(self, h: int, gen) -> int:
        d, svf = getattr(gen, "diode", None), getattr(gen, "sky_view", None)
        try:
            if d is not None:
                self.set_diode(h, d)
            if svf is not None:
                self.set_sky(h, svf)
        except Pv3dError:
            self.release_generator(h)
            raise
        return h

    def set_sky(self, gen_h: int, svf):
        """Per-cell sky view factors [n_cells] scaling each cell's diffuse, or None to detach them."""
        a = None if svf is None else _c(svf, np.float64).reshape(-1)
        _check(lib().pv3d_generator_set_sky(self.h, gen_h, _ptr(a)), self.h)

    def sky_view(self, scene_h: int, gen_h: int, gen, dirs, map_n: int, k: int, tile: int = 0) -> np.ndarray:
        """Sky view factor of every cell over the sky directions dirs [n, 3] (computed on the GPU)."""
        d = _c(dirs, np.float64).reshape(-1, 3)
        out = np.zeros(gen.n_cells)
        p = self.params(map_n, k, tile=tile)
        _check(lib().pv3d_sky_view(self.h, scene_h, gen_h, _ptr(d), d.shape[0], ctypes.byref(p), _ptr(out)), self.h)
        return out

    def set_diode(self, gen_h: int, d):
        """Single-diode cell model for the generator: d = (Isc_ref, G_ref, I0, a, Rs, Rsh, Vb), or None
        for ideal bypass-diode strings."""
        if d is None:
            _check(lib().pv3d_generator_set_diode(self.h, gen_h, None), self.h)
            return
        v = [float(x) for x in np.asarray(d, np.float64).reshape(-1)]
        if len(v) != 7:
            raise ValueError("diode parameters: Isc_ref, G_ref, I0, a, Rs, Rsh, Vb")
        dd = Diode(*v)
        _check(lib().pv3d_generator_set_diode(self.h, gen_h, ctypes.byref(dd)), self.h)

    def release_generator(self, h: int):
        _check(lib().pv3d_generator_release(self.h, h), self.h)

    @staticmethod
    def params(map_n: int, k: int, export_depth=False, export_bits=False, tile: int = 0,
               separate_test=False, full_raster=False, bin_limit: int = 0) -> Params:
        return Params(map_n, k, (EXPORT_DEPTH if export_depth else 0) | (EXPORT_BITS if export_bits else 0)
                      | (SEPARATE_TEST if separate_test else 0) | (FULL_RASTER if full_raster else 0), tile,
                      bin_limit, 0)

    def evaluate(self, scene_h: int, gen_h: int, gen, sweep, map_n: int, k: int, export_depth=False,
                 export_bits=False, tile: int = 0, separate_test=False, full_raster=False,
                 bin_limit: int = 0) -> Result:
        """Host outputs (synchronous)."""
        s = _c(sweep.sun_xyz, np.float64)
        dni, dp, dt = (_c(a, np.float64) for a in (sweep.dni, sweep.d_poa, sweep.dt_h))
        n = s.shape[0]
        cells = gen.n_cells
        words = (k * k + 31) // 32
        counts = np.zeros((n, cells), np.uint32)
        pw, pr, en = np.zeros(n), np.zeros(n), np.zeros(2)
        maps = np.zeros((n, map_n, map_n), np.uint32) if export_depth else None
        bits = np.zeros((n, cells, words), np.uint32) if export_bits else None
        out = Outputs(_ptr(counts), _ptr(pw), _ptr(pr), _ptr(en), _ptr(maps), _ptr(bits), 0)
        p = self.params(map_n, k, export_depth, export_bits, tile, separate_test, full_raster, bin_limit)
        _check(lib().pv3d_evaluate(self.h, scene_h, gen_h, _ptr(s), _ptr(dni), _ptr(dp), _ptr(dt), n,
                                   ctypes.byref(p), ctypes.byref(out), None), self.h)
        return Result(counts, pw, pr, en, maps, bits)

    def evaluate_device(self, scene_h: int, gen_h: int, gen, sweep, map_n: int, k: int, stream=None,
                        counts=None, tile: int = 0, separate_test=False, full_raster=False,
                        bin_limit: int = 0) -> Result:
        """Device outputs as torch tensors, asynchronous on `stream` (default: torch's current stream)."""
        import torch
        s = _c(sweep.sun_xyz, np.float64)
        dni, dp, dt = (_c(a, np.float64) for a in (sweep.dni, sweep.d_poa, sweep.dt_h))
        n = s.shape[0]
        dev = torch.device("cuda", torch.cuda.current_device())
        pw = torch.empty(n, dtype=torch.float64, device=dev)
        pr = torch.empty(n, dtype=torch.float64, device=dev)
        en = torch.empty(2, dtype=torch.float64, device=dev)
        out = Outputs(_ptr(counts), _ptr(pw), _ptr(pr), _ptr(en), None, None, 1)
        p = self.params(map_n, k, tile=tile, separate_test=separate_test, full_raster=full_raster, bin_limit=bin_limit)
        st = stream if stream is not None else torch.cuda.current_stream()
        with _Ordered(st) as hs:
            _check(lib().pv3d_evaluate(self.h, scene_h, gen_h, _ptr(s), _ptr(dni), _ptr(dp), _ptr(dt), n,
                                       ctypes.byref(p), ctypes.byref(out), hs), self.h)
        return Result(counts, pw, pr, en)

    def evaluate_noalloc(self, scene_h: int, gen_h: int, gen, sweep, map_n: int, k: int, counts, power, power_ref,
                         energy, stream=None, tile: int = 0, bin_limit: int = 0, separate_test=False) -> Result:
        """pv3d_evaluate_noalloc into caller-owned device tensors (counts may be None), asynchronous on
        `stream` (default: torch's current stream); the library allocates nothing for the call."""
        import torch
        s = _c(sweep.sun_xyz, np.float64)
        dni, dp, dt = (_c(a, np.float64) for a in (sweep.dni, sweep.d_poa, sweep.dt_h))
        out = Outputs(_ptr(counts), _ptr(power), _ptr(power_ref), _ptr(energy), None, None, 1)
        p = self.params(map_n, k, tile=tile, separate_test=separate_test, bin_limit=bin_limit)
        st = stream if stream is not None else torch.cuda.current_stream()
        with _Ordered(st) as hs:
            _check(lib().pv3d_evaluate_noalloc(self.h, scene_h, gen_h, _ptr(s), _ptr(dni), _ptr(dp), _ptr(dt),
                                               s.shape[0], ctypes.byref(p), ctypes.byref(out), hs), self.h)
        return Result(counts, power, power_ref, energy)

    # ------------------------------------------------------------------
    # batched form
    # ------------------------------------------------------------------
    def _job(self, spec, device: bool, keep: list) -> Job:
        """spec: dict with scene, gen (handles), generator, sweep, map_n, k and optional tile,
        bin_limit, full_raster. Host outputs are numpy arrays; device outputs torch tensors."""
        sw, g = spec["sweep"], spec["generator"]
        arrs = [_c(sw.sun_xyz, np.float64), _c(sw.dni, np.float64), _c(sw.d_poa, np.float64),
                _c(sw.dt_h, np.float64)]
        keep.append(arrs)
        n = arrs[0].shape[0]
        if device:
            # no fill: the library writes every element (the batched form clears the outputs on its
            # stream first; the serving loop clears each sun's counts and writes every power), and a
            # fill on torch's stream would not be ordered before the serving loop's writes
            import torch
            dev = torch.device("cuda", torch.cuda.current_device())
            counts = torch.empty((n, g.n_cells), dtype=torch.int32, device=dev) if spec.get("counts", True) else None
            pw = torch.empty(n, dtype=torch.float64, device=dev)
            pr = torch.empty(n, dtype=torch.float64, device=dev)
            en = torch.empty(2, dtype=torch.float64, device=dev)
        else:
            counts = np.zeros((n, g.n_cells), np.uint32) if spec.get("counts", True) else None
            pw, pr, en = np.zeros(n), np.zeros(n), np.zeros(2)
        res = Result(counts, pw, pr, en)
        keep.append(res)
        p = self.params(spec["map_n"], spec["k"], tile=spec.get("tile", 0), full_raster=spec.get("full_raster", False),
                        bin_limit=spec.get("bin_limit", 0))
        out = Outputs(_ptr(counts), _ptr(pw), _ptr(pr), _ptr(en), None, None, 1 if device else 0)
        return Job(spec["scene"], spec["gen"], _ptr(arrs[0]), _ptr(arrs[1]), _ptr(arrs[2]), _ptr(arrs[3]), n, p, out)

    def evaluate_batched(self, specs, device: bool = False, stream=None):
        """Every job of `specs` (see _job) in one persistent launch; one Result per job."""
        keep: list = []
        jobs = (Job * len(specs))(*[self._job(sp, device, keep) for sp in specs])
        results = [r for r in keep if isinstance(r, Result)]
        st = None
        if device:
            import torch
            st = ctypes.c_void_p((stream if stream is not None else torch.cuda.current_stream()).cuda_stream)
        _check(lib().pv3d_evaluate_batched(self.h, jobs, len(specs), st), self.h)
        return results

    def autotune(self, spec, n_probe: int = 8):
        """(tile, bin_limit, best probe milliseconds) the autotuner picks for one job."""
        keep: list = []
        job = self._job(dict(spec, counts=False), False, keep)
        ms = _f64()
        _check(lib().pv3d_autotune(self.h, ctypes.byref(job), n_probe, ctypes.byref(ms)), self.h)
        return job.params.tile, job.params.bin_limit, ms.value

    def tuning_cache(self, mode: int, path: Optional[str] = None):
        """The autotuner's cache: TUNE_SAVE writes it to the JSON file at path, TUNE_LOAD adds a
        saved file's classes, TUNE_CLEAR empties it."""
        _check(lib().pv3d_autotune_cache(self.h, path.encode() if path is not None else None, mode), self.h)

    def batch_limits(self, max_slots: int = 0, slot_records: int = 0, any_xcd: bool = False):
        _check(lib().pv3d_batch_limits(self.h, max_slots, slot_records, BATCH_ANY_XCD if any_xcd else 0), self.h)

    def path_stats(self) -> dict:
        """Work counts of the last per-sun evaluation (waits for it to end)."""
        a = (_i64 * 4)()
        _check(lib().pv3d_path_stats(self.h, ctypes.byref(a)), self.h)
        return dict(zip(("suns", "records", "large", "pairs"), list(a)))

    def batch_stats(self) -> dict:
        a = (_i64 * 7)()
        _check(lib().pv3d_batch_stats(self.h, ctypes.byref(a)), self.h)
        return dict(zip(("items", "units", "redone", "workgroups", "slots", "launch_us", "xcd_groups"), list(a)))

    # ------------------------------------------------------------------
    # serving loop
    # ------------------------------------------------------------------
    def submit(self, spec, device: bool = False) -> int:
        """Submit one job (see _job) to the serving loop; returns its ticket. The Result
        (host arrays, filled when the job ends) is kept until wait()."""
        keep: list = []
        job = self._job(spec, device, keep)
        t = _u64()
        _check(lib().pv3d_submit(self.h, ctypes.byref(job), ctypes.byref(t)), self.h)
        if not hasattr(self, "_tickets"):
            self._tickets = {}
        self._tickets[t.value] = [r for r in keep if isinstance(r, Result)][0]
        return t.value

    def poll(self, ticket: int) -> bool:
        d = _i32()
        _check(lib().pv3d_poll(self.h, ticket, ctypes.byref(d)), self.h)
        return bool(d.value)

    def wait(self, ticket: int) -> Result:
        """Block until the job ends; its Result (raises Pv3dError if cancelled or failed)."""
        res = self._tickets.pop(ticket, None)
        _check(lib().pv3d_wait(self.h, ticket), self.h)
        return res

    def cancel(self, ticket: int):
        _check(lib().pv3d_cancel(self.h, ticket), self.h)

    def serve_stats(self) -> dict:
        a = (_i64 * 4)()
        _check(lib().pv3d_serve_stats(self.h, ctypes.byref(a)), self.h)
        return dict(zip(("jobs_done", "launches", "items", "pending"), list(a)))
