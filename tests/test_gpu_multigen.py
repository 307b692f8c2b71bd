"""Many generators in one scene on the GPU (needs an MI355X): the scene is
loaded once, every generator is defined against it, and all generators go
through one persistent launch, one job per generator (Sec. 3.3's case). Counts
and shaded flags bit-exact against the oracle; powers and energies within 1e-6
relative; the batched launch identical to the per-sun path, generator by
generator."""
import numpy as np
import pytest

from paper_1410_5780_amd import workloads as W
from tests.test_gpu_parity import REL, ctx, _say  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu


def _specs(ctx, ws):
    sh = ctx.load_scene(ws[0].scene)
    return sh, [dict(scene=sh, gen=ctx.define_generator(w.gen), generator=w.gen, sweep=w.sweep, map_n=w.map_n,
                     k=w.k) for w in ws]


def _release(ctx, sh, specs):
    for sp in specs:
        ctx.release_generator(sp["gen"])
    ctx.release_scene(sh)


def _against_oracle(w, got, ref):
    assert ref.outside == 0
    assert np.array_equal(np.asarray(got.counts), ref.counts), w.name
    np.testing.assert_allclose(np.asarray(got.power), ref.power, rtol=REL, atol=0)
    np.testing.assert_allclose(np.asarray(got.power_ref), ref.power_ref, rtol=REL, atol=0)
    np.testing.assert_allclose(np.asarray(got.energy), ref.energy, rtol=REL, atol=0)


def test_small_stadium_every_generator(ctx, oracle_lib):
    """Ten generators sharing one scene: per-sun path (with pictures and flags) and one
    batched launch over all ten, both against the oracle."""
    ws = W.c7_stadium_small()
    sh, specs = _specs(ctx, ws)
    try:
        batched = ctx.evaluate_batched(specs)
        total = 0
        for w, sp, b in zip(ws, specs, batched):
            ref = oracle_lib.evaluate(w.scene, w.gen, w.sweep, w.map_n, w.k, export_maps=True, export_bits=True)
            got = ctx.evaluate(sh, sp["gen"], w.gen, w.sweep, w.map_n, w.k, export_depth=True, export_bits=True)
            _against_oracle(w, got, ref)
            assert np.array_equal(got.maps, ref.maps) and np.array_equal(got.bits, ref.bits), w.name
            _against_oracle(w, b, ref)
            for f in ("counts", "power", "power_ref", "energy"):
                assert np.array_equal(np.asarray(getattr(b, f)), getattr(got, f)), (w.name, f)
            total += int(ref.counts.sum())
        _say(f"[multigen] small stadium: {len(ws)} generators identical, shaded {total}")
        assert total > 10000
    finally:
        _release(ctx, sh, specs)


def test_stadium_full_size_sampled_suns(ctx, oracle_lib):
    """88 generators of 14 x 4 modules, N = 4096, k = 8, every 800th sun of the year: one
    batched launch over all 88 against the oracle, generator by generator."""
    yr = W.year_sweep()
    ws = W.c7_stadium(sweep=yr.subset(np.arange(0, yr.n, 800)))
    sh, specs = _specs(ctx, ws)
    try:
        batched = ctx.evaluate_batched(specs)
        st = ctx.batch_stats()
        _say(f"[multigen] stadium: {len(ws)} jobs, {ws[0].sweep.n} suns each, stats {st}")
        total = 0
        for w, b in zip(ws, batched):
            ref = oracle_lib.evaluate(w.scene, w.gen, w.sweep, w.map_n, w.k, threads=0)
            _against_oracle(w, b, ref)
            total += int(ref.counts.sum())
        _say(f"[multigen] stadium: all 88 generators match the oracle, shaded {total}")
        assert total > 0
    finally:
        _release(ctx, sh, specs)


def test_stadium_batched_equals_per_sun_path(ctx):
    """Every 97th sun of the year for all 88 generators: one launch, each job bit-identical
    to pv3d_evaluate of its generator."""
    yr = W.year_sweep()
    ws = W.c7_stadium(sweep=yr.subset(np.arange(0, yr.n, 97)))
    sh, specs = _specs(ctx, ws)
    try:
        batched = ctx.evaluate_batched(specs)
        for w, sp, b in zip(ws, specs, batched):
            a = ctx.evaluate(sh, sp["gen"], w.gen, w.sweep, w.map_n, w.k)
            for f in ("counts", "power", "power_ref", "energy"):
                assert np.array_equal(np.asarray(getattr(b, f)), getattr(a, f)), (w.name, f)
        _say(f"[multigen] stadium every 97th sun: batched identical to the per-sun path for {len(ws)} generators")
    finally:
        _release(ctx, sh, specs)
