"""Trackers on the GPU against the oracle (needs an MI355X): modules posed for
every sun on the device, then the same path as fixed modules. Depth pictures,
shaded flags and counts bit-exact; powers and energies within 1e-6 relative."""
import numpy as np
import pytest

from paper_1410_5780_amd import workloads as W
from tests.test_gpu_parity import compare, ctx, _say  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", [1, 2])
def test_tracker_pair_full(ctx, oracle_lib, kind):
    got, ref = compare(ctx, oracle_lib, W.tracker_pair(kind=kind))
    assert int(got.counts.sum()) > 2000            # the pair shades itself on some suns


def test_tracker_plant_full_size_sampled_suns(ctx, oracle_lib):
    """The two-axis plant on terrain with its pylon, every 200th sun of the year, N = 4096, k = 8."""
    yr = W.year_sweep()
    w = W.c6_tracker_plant(sweep=yr.subset(np.arange(0, yr.n, 200)))
    compare(ctx, oracle_lib, w, maps=False, bits=False, threads=0)


def test_tracker_rows_sampled_suns(ctx, oracle_lib):
    """One-axis tracker rows with 50 pylons, every 300th sun of the year, N = 4096, k = 8."""
    yr = W.year_sweep()
    w = W.c2_tracker_rows(sweep=yr.subset(np.arange(0, yr.n, 300)))
    compare(ctx, oracle_lib, w, maps=False, bits=False, threads=0)


def test_tracked_generator_errors(ctx):
    from paper_1410_5780_amd import pv3d
    w = W.tracker_pair(kind=2)
    g = w.gen

    def define(**kw):
        import dataclasses
        return ctx.define_generator(dataclasses.replace(g, **kw))

    bad_kind = g.trackers.copy()
    bad_kind[0, 0] = 3
    tilted = g.trackers.copy()
    tilted[0, 4:7] = [0.0, 0.8, 0.6]
    short = g.trackers.copy()
    short[0, 4:7] = [0.0, 0.5, 0.0]
    wrong_index = g.module_tracker.copy()
    wrong_index[0] = 2
    for kw in (dict(trackers=bad_kind), dict(trackers=tilted), dict(trackers=short),
               dict(module_tracker=wrong_index)):
        with pytest.raises(pv3d.Pv3dError) as e:
            define(**kw)
        assert e.value.code == pv3d.EINVAL
    # the serving loop refuses tracked generators
    sh, gh = ctx.load_scene(w.scene), ctx.define_generator(g)
    spec = dict(scene=sh, gen=gh, generator=g, sweep=w.sweep, map_n=w.map_n, k=w.k)
    with pytest.raises(pv3d.Pv3dError) as e:
        ctx.submit(spec)
    assert e.value.code == pv3d.EINVAL


def test_batched_trackers_match_the_per_sun_path(ctx):
    """Tracked and fixed generators in one persistent launch: every job bit-identical to pv3d_evaluate."""
    yr = W.year_sweep()
    ws = [W.tracker_pair(kind=2), W.tracker_pair(kind=1),
          W.c6_tracker_plant(sweep=yr.subset(np.arange(0, yr.n, 97))), W.c1_tiny(d_poa=100.0)]
    specs = [dict(scene=ctx.load_scene(w.scene), gen=ctx.define_generator(w.gen), generator=w.gen, sweep=w.sweep,
                  map_n=w.map_n, k=w.k) for w in ws]
    got = ctx.evaluate_batched(specs)
    for w, sp, b in zip(ws, specs, got):
        a = ctx.evaluate(sp["scene"], sp["gen"], w.gen, w.sweep, w.map_n, w.k)
        assert np.array_equal(np.asarray(b.counts), a.counts), w.name
        assert np.array_equal(np.asarray(b.power), a.power), w.name
        assert np.array_equal(np.asarray(b.energy), a.energy), w.name
        _say(f"[trackers] batched {w.name}: identical, shaded {int(a.counts.sum())}")


def test_tracker_pair_most_samples_per_cell(ctx, oracle_lib):
    """Two-axis trackers at k = 255 (65,025 samples per cell) on low winter suns, when the southern
    tracker shades the northern one: each sun's posed modules, flags and counts as in the oracle."""
    sw = W.make_sweep(W.LAT_DEG, [355], [8.5, 9.5, 14.5, 15.5], up_only=True)
    got, ref = compare(ctx, oracle_lib, W.tracker_pair(kind=2, k=255, sweep=sw), maps=False, bits=True)
    assert (ref.counts.sum(axis=1) > 0).sum() >= 2
