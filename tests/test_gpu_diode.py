"""The single-diode electrical model on the GPU against the oracle (needs an
MI355X): the shading path is unchanged (counts bit-exact), and powers and
energies from the per-string maximum power search agree within 1e-6 relative.
The per-sun path, the batched launch and the serving loop give identical
results for the same generator."""
import dataclasses

import numpy as np
import pytest

from paper_1410_5780_amd import workloads as W
from tests.test_gpu_parity import REL, ctx, _say  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu

D = W.DIODE_CELL


def _diode(w, d=D):
    return dataclasses.replace(w, gen=dataclasses.replace(w.gen, diode=np.asarray(d, np.float64)))


def _compare(ctx, oracle_lib, w):
    _say(f"[diode] {w.name}: cells={w.gen.n_cells} strings={w.gen.n_string} suns={w.sweep.n} N={w.map_n} k={w.k}")
    sh, gh = ctx.load_scene(w.scene), ctx.define_generator(w.gen)
    try:
        got = ctx.evaluate(sh, gh, w.gen, w.sweep, w.map_n, w.k)
    finally:
        ctx.release_scene(sh)
        ctx.release_generator(gh)
    ref = oracle_lib.evaluate(w.scene, w.gen, w.sweep, w.map_n, w.k)
    assert ref.outside == 0
    assert np.array_equal(got.counts, ref.counts)
    np.testing.assert_allclose(got.power, ref.power, rtol=REL, atol=0)
    np.testing.assert_allclose(got.power_ref, ref.power_ref, rtol=REL, atol=0)
    np.testing.assert_allclose(got.energy, ref.energy, rtol=REL, atol=0)
    up = ref.power_ref > 0
    worst = float(np.max(np.abs(got.power[up] - ref.power[up]) / ref.power_ref[up])) if up.any() else 0.0
    _say(f"[diode] {w.name}: ok, loss {got.loss:.6f} (oracle {ref.loss:.6f}), worst relative power gap {worst:.2e}")
    return got, ref


def test_c1_tiny_diode(ctx, oracle_lib):
    got, ref = _compare(ctx, oracle_lib, _diode(W.c1_tiny(d_poa=100.0)))
    assert got.energy[0] < got.energy[1]


def test_row_plant_sampled_suns_diode(ctx, oracle_lib):
    """C2 (20 strings of 20 modules, 1,200 cells each) on every 150th sun of the year."""
    yr = W.year_sweep()
    _compare(ctx, oracle_lib, _diode(W.c2_row_plant(sweep=yr.subset(np.arange(0, yr.n, 150)))))


def test_long_string_read_from_device_memory(ctx, oracle_lib):
    """A string of 80 modules (4,800 cells) is too long to stage in LDS: its counts are read
    from device memory on every evaluation of the string."""
    w = W.c2_row_plant(sweep=W.make_sweep(W.LAT_DEG, [355, 20], np.arange(7, 18)), n_pylons=50)
    g = dataclasses.replace(w.gen, module_string=(np.arange(w.gen.n_mod) // 80).astype(np.int32), diode=D)
    _compare(ctx, oracle_lib, dataclasses.replace(w, gen=g, name="c2_strings_of_80"))


def test_random_tiny_diode(ctx, oracle_lib):
    for seed in range(3):
        _compare(ctx, oracle_lib, _diode(W.random_tiny(100 + seed)))


def test_trackers_with_diode(ctx, oracle_lib):
    _compare(ctx, oracle_lib, _diode(W.tracker_pair(kind=2)))


def _served_in_own_context(ws, specs):
    """The jobs served by a context of their own (the serving loop does not start in a
    context whose per-sun path has run)."""
    from paper_1410_5780_amd import pv3d
    with pv3d.Context(0) as sc:
        own = [dict(sp, scene=sc.load_scene(w.scene), gen=sc.define_generator(sp["generator"]))
               for w, sp in zip(ws, specs)]
        tickets = [sc.submit(sp) for sp in own]
        return [sc.wait(t) for t in tickets]


def test_diode_batched_and_served_equal_per_sun(ctx):
    yr = W.year_sweep()
    ws = [_diode(W.c2_row_plant(sweep=yr.subset(np.arange(0, yr.n, 211)))), _diode(W.c1_tiny(d_poa=100.0)),
          W.c1_tiny(d_poa=100.0)]
    specs = [dict(scene=ctx.load_scene(w.scene), gen=ctx.define_generator(w.gen), generator=w.gen, sweep=w.sweep,
                  map_n=w.map_n, k=w.k) for w in ws]
    batched = ctx.evaluate_batched(specs)
    served = _served_in_own_context(ws, specs)
    for w, sp, b, sv in zip(ws, specs, batched, served):
        a = ctx.evaluate(sp["scene"], sp["gen"], w.gen, w.sweep, w.map_n, w.k)
        for f in ("counts", "power", "power_ref", "energy"):
            assert np.array_equal(np.asarray(getattr(b, f)), getattr(a, f)), (w.name, f, "batched")
            assert np.array_equal(np.asarray(getattr(sv, f)), getattr(a, f)), (w.name, f, "served")
        _say(f"[diode] {w.name}: batched and served identical to the per-sun path")


def test_set_diode_errors_and_reset(ctx):
    from paper_1410_5780_amd import pv3d
    w = W.c1_tiny(d_poa=100.0)
    sh, gh = ctx.load_scene(w.scene), ctx.define_generator(w.gen)
    try:
        ideal = ctx.evaluate(sh, gh, w.gen, w.sweep, w.map_n, w.k)
        for i, bad in ((0, 0.0), (1, -1.0), (2, 0.0), (3, float("nan")), (4, -1e-3), (5, 0.0), (6, -0.1),
                       (2, float("inf"))):
            d = D.copy()
            d[i] = bad
            with pytest.raises(pv3d.Pv3dError) as e:
                ctx.set_diode(gh, d)
            assert e.value.code == pv3d.EINVAL, (i, bad)
        with pytest.raises(pv3d.Pv3dError) as e:
            ctx.set_diode(gh + 12345, D)
        assert e.value.code == pv3d.ENOENT
        ctx.set_diode(gh, D)
        dio = ctx.evaluate(sh, gh, w.gen, w.sweep, w.map_n, w.k)
        assert np.array_equal(dio.counts, ideal.counts) and not np.array_equal(dio.power, ideal.power)
        ctx.set_diode(gh, None)
        back = ctx.evaluate(sh, gh, w.gen, w.sweep, w.map_n, w.k)
        assert np.array_equal(back.power, ideal.power) and np.array_equal(back.energy, ideal.energy)
    finally:
        ctx.release_scene(sh)
        ctx.release_generator(gh)


def test_most_samples_per_cell_diode(ctx, oracle_lib):
    """k = 255 (65,025 samples per cell): too many shaded-count levels for one solve per level, so
    every string takes the per-lane form."""
    w = W.random_tiny(81, n_boxes=6, n_loose=6, n_mod_side=2, map_n=256, k=255, n_sun=2)
    got, ref = _compare(ctx, oracle_lib, _diode(w))
    assert ref.counts.sum() > 100000 and got.energy[0] < got.energy[1]
