"""Diffuse shading on the GPU against the oracle (needs an MI355X): sky view
factors computed by pv3d_sky_view (every sky direction through the shading
path, then a per-cell reduction on the device) are bit-identical to the
oracle's; with the factors attached, powers and energies agree with the oracle
(ideal strings and the single-diode model), and the batched and served forms
with the per-sun path."""
import dataclasses

import numpy as np
import pytest

from paper_1410_5780_amd import workloads as W
from tests.test_gpu_parity import REL, ctx, _say  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu


def _sky(ctx, oracle_lib, w, n_dir, map_n, k):
    d = W.sky_directions(n_dir)
    sh, gh = ctx.load_scene(w.scene), ctx.define_generator(w.gen)
    try:
        got = ctx.sky_view(sh, gh, w.gen, d, map_n, k)
    finally:
        ctx.release_scene(sh)
        ctx.release_generator(gh)
    ref = oracle_lib.sky_view(w.scene, w.gen, d, map_n, k)
    bad = np.nonzero(got != ref)[0]
    assert bad.size == 0, f"{w.name}: {bad.size} cells differ, first {bad[:5]}: {got[bad[:5]]} vs {ref[bad[:5]]}"
    _say(f"[sky] {w.name}: {n_dir} directions, N={map_n}, k={k}: identical; svf {ref.min():.4f}..{ref.max():.4f}")
    return ref


def test_sky_view_c1(ctx, oracle_lib):
    svf = _sky(ctx, oracle_lib, W.c1_tiny(), 1024, 1024, 8)
    assert svf.min() < 0.99


def test_sky_view_random_tiny(ctx, oracle_lib):
    for seed in range(3):
        w = W.random_tiny(200 + seed)
        _sky(ctx, oracle_lib, w, 257, w.map_n, w.k)


def test_sky_view_row_plant(ctx, oracle_lib):
    """C2's rows and pylons, 145 directions at N = 4096, k = 8."""
    w = W.c2_row_plant(sweep=W.make_sweep(W.LAT_DEG, [172], [12.0]))
    svf = _sky(ctx, oracle_lib, w, 145, w.map_n, w.k)
    assert svf.min() < 0.9          # the rows hide part of each other's sky


def test_evaluate_with_sky_view(ctx, oracle_lib):
    """C1 and C2 (every 200th sun) with their sky view factors attached, ideal strings and the
    single-diode model, against the oracle."""
    yr = W.year_sweep()
    c1 = W.c1_tiny(d_poa=100.0)
    c2 = W.c2_row_plant(sweep=yr.subset(np.arange(0, yr.n, 200)))
    # any factors in [0, 1] exercise the loss path: the oracle's for C1, seeded ones for C2
    rng = np.random.default_rng(11)
    for w, svf in ((c1, oracle_lib.sky_view(c1.scene, c1.gen, W.sky_directions(512), c1.map_n, c1.k)),
                   (c2, rng.uniform(0.6, 1.0, c2.gen.n_cells))):
        for diode in (None, W.DIODE_CELL):
            g = dataclasses.replace(w.gen, sky_view=svf, diode=diode)
            sh, gh = ctx.load_scene(w.scene), ctx.define_generator(g)
            try:
                got = ctx.evaluate(sh, gh, g, w.sweep, w.map_n, w.k)
            finally:
                ctx.release_scene(sh)
                ctx.release_generator(gh)
            ref = oracle_lib.evaluate(w.scene, g, w.sweep, w.map_n, w.k)
            assert np.array_equal(got.counts, ref.counts)
            np.testing.assert_allclose(got.power, ref.power, rtol=REL, atol=0)
            np.testing.assert_allclose(got.power_ref, ref.power_ref, rtol=REL, atol=0)
            np.testing.assert_allclose(got.energy, ref.energy, rtol=REL, atol=0)
            if diode is None:
                assert np.array_equal(got.power, ref.power) and np.array_equal(got.energy, ref.energy)
            _say(f"[sky] {w.name} diode={diode is not None}: loss {got.loss:.6f} (oracle {ref.loss:.6f})")


def test_sky_view_batched_and_served_equal_per_sun(ctx):
    yr = W.year_sweep()
    w = W.c2_row_plant(sweep=yr.subset(np.arange(0, yr.n, 311)))
    svf = np.random.default_rng(12).uniform(0.6, 1.0, w.gen.n_cells)
    gens = [dataclasses.replace(w.gen, sky_view=svf), dataclasses.replace(w.gen, sky_view=svf, diode=W.DIODE_CELL)]
    sh = ctx.load_scene(w.scene)
    specs = [dict(scene=sh, gen=ctx.define_generator(g), generator=g, sweep=w.sweep, map_n=w.map_n, k=w.k)
             for g in gens]
    batched = ctx.evaluate_batched(specs)
    from paper_1410_5780_amd import pv3d
    with pv3d.Context(0) as other:          # the serving loop starts in a context of its own
        sh2 = other.load_scene(w.scene)
        own = [dict(sp, scene=sh2, gen=other.define_generator(g)) for g, sp in zip(gens, specs)]
        served = [other.wait(other.submit(sp)) for sp in own]
    for g, sp, b, sv in zip(gens, specs, batched, served):
        a = ctx.evaluate(sh, sp["gen"], g, w.sweep, w.map_n, w.k)
        for f in ("counts", "power", "power_ref", "energy"):
            assert np.array_equal(np.asarray(getattr(b, f)), getattr(a, f)), (f, "batched")
            assert np.array_equal(np.asarray(getattr(sv, f)), getattr(a, f)), (f, "served")
    _say("[sky] batched and served identical to the per-sun path")


def test_sky_errors(ctx):
    from paper_1410_5780_amd import pv3d
    w = W.c1_tiny(d_poa=100.0)
    sh, gh = ctx.load_scene(w.scene), ctx.define_generator(w.gen)
    try:
        plain = ctx.evaluate(sh, gh, w.gen, w.sweep, w.map_n, w.k)
        for bad in (1.5, -0.1, float("nan")):
            v = np.ones(w.gen.n_cells)
            v[7] = bad
            with pytest.raises(pv3d.Pv3dError) as e:
                ctx.set_sky(gh, v)
            assert e.value.code == pv3d.EINVAL
        below = W.sky_directions(8)
        below[3, 2] = -below[3, 2]
        with pytest.raises(pv3d.Pv3dError) as e:
            ctx.sky_view(sh, gh, w.gen, below, 256, 4)
        assert e.value.code == pv3d.EINVAL
        with pytest.raises(pv3d.Pv3dError) as e:
            ctx.set_sky(gh + 999, np.ones(w.gen.n_cells))
        assert e.value.code == pv3d.ENOENT
        ctx.set_sky(gh, np.full(w.gen.n_cells, 0.5))
        half = ctx.evaluate(sh, gh, w.gen, w.sweep, w.map_n, w.k)
        assert np.all(half.power <= plain.power) and np.array_equal(half.power_ref, plain.power_ref)
        ctx.set_sky(gh, None)
        back = ctx.evaluate(sh, gh, w.gen, w.sweep, w.map_n, w.k)
        assert np.array_equal(back.power, plain.power)
    finally:
        ctx.release_scene(sh)
        ctx.release_generator(gh)
    t = W.tracker_pair(kind=2)
    sh, gh = ctx.load_scene(t.scene), ctx.define_generator(t.gen)
    try:
        with pytest.raises(pv3d.Pv3dError) as e:
            ctx.set_sky(gh, np.ones(t.gen.n_cells))
        assert e.value.code == pv3d.EINVAL
        with pytest.raises(pv3d.Pv3dError) as e:
            ctx.sky_view(sh, gh, t.gen, W.sky_directions(16), 256, 4)
        assert e.value.code == pv3d.EINVAL
    finally:
        ctx.release_scene(sh)
        ctx.release_generator(gh)


def test_sky_view_edge_directions(ctx, oracle_lib):
    """One direction only, directions a hair above the horizon (a near-horizontal view), and
    k = 1: the factors stay bit-identical to the oracle's."""
    w = W.c1_tiny()
    low = np.array([[np.cos(e) * np.cos(a), np.cos(e) * np.sin(a), np.sin(e)]
                    for e in (0.01, 0.05) for a in [*np.linspace(0.0, 2.0 * np.pi, 7, endpoint=False), 1.5 * np.pi]])
    cases = [(np.array([[0.0, 0.0, 1.0]]), 512, 4), (low, 1024, 8), (W.sky_directions(64), 256, 1)]
    sh, gh = ctx.load_scene(w.scene), ctx.define_generator(w.gen)
    try:
        for dirs, n, k in cases:
            got = ctx.sky_view(sh, gh, w.gen, dirs, n, k)
            ref = oracle_lib.sky_view(w.scene, w.gen, dirs, n, k)
            assert np.array_equal(got, ref), (dirs.shape[0], n, k)
            _say(f"[sky] {dirs.shape[0]} directions, N={n}, k={k}: identical, svf {ref.min():.4f}..{ref.max():.4f}")
    finally:
        ctx.release_scene(sh)
        ctx.release_generator(gh)


def test_sky_view_most_samples_per_cell(ctx, oracle_lib):
    """k = 255 (65,025 samples per cell): each direction's shaded share is a count over k^2 near its
    largest; the factors stay bit-identical to the oracle's."""
    w = W.random_tiny(81, n_boxes=6, n_loose=6, n_mod_side=2, map_n=256, k=255, n_sun=2)
    svf = _sky(ctx, oracle_lib, w, 8, 256, 255)
    assert svf.min() < 0.9
