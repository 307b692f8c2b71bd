"""Batched form (one persistent launch over every (job, sun) item) against the
per-sun path and the CPU oracle, through the C ABI (needs an MI355X).

The persistent kernel runs the same per-unit code as the per-sun kernels, so
counts, powers and energies must be identical, bit for bit, job by job.
"""
import sys

import numpy as np
import pytest

from paper_1410_5780_amd import workloads as W
from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_1410_5780_amd import pv3d
    c = pv3d.Context(0)
    yield c
    c.close()


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _spec(ctx, w, **kw):
    d = dict(scene=ctx.load_scene(w.scene), gen=ctx.define_generator(w.gen), generator=w.gen, sweep=w.sweep,
             map_n=w.map_n, k=w.k)
    d.update(kw)
    return d


def _same(a, b, what):
    assert np.array_equal(np.asarray(a.counts), np.asarray(b.counts)), f"{what}: counts differ"
    assert np.array_equal(np.asarray(a.power), np.asarray(b.power)), f"{what}: power differs"
    assert np.array_equal(np.asarray(a.power_ref), np.asarray(b.power_ref)), f"{what}: power_ref differs"
    assert np.array_equal(np.asarray(a.energy), np.asarray(b.energy)), f"{what}: energy differs"


def _plain(ctx, sp):
    return ctx.evaluate(sp["scene"], sp["gen"], sp["generator"], sp["sweep"], sp["map_n"], sp["k"],
                        tile=sp.get("tile", 0) or 64, full_raster=sp.get("full_raster", False),
                        bin_limit=sp.get("bin_limit", 0))


def _uneven_jobs():
    """Tiny cases of different sizes, tiles, k and map sizes, with suns below the horizon mixed in."""
    ws = []
    for i, (n, k, side, boxes, loose) in enumerate([(200, 3, 3, 10, 40), (130, 4, 2, 3, 10), (333, 5, 3, 12, 60),
                                                    (64, 16, 2, 0, 5), (257, 1, 3, 8, 30), (96, 2, 1, 4, 4)]):
        w = W.random_tiny(60 + i, n_boxes=boxes, n_loose=loose, n_mod_side=side, map_n=n, k=k, n_sun=7)
        ws.append(w)
    c1 = W.c1_tiny(d_poa=100.0)
    ws.append(c1)                                   # 24 hours: 9 above the horizon
    return ws


def test_batched_matches_per_sun_path_and_oracle(ctx, oracle_lib):
    ws = _uneven_jobs()
    specs = [_spec(ctx, w, tile=(32 if i % 2 else 64)) for i, w in enumerate(ws)]
    _say(f"[batched] {len(specs)} jobs, {sum(int((w.sweep.sun_xyz[:, 2] > 0).sum()) for w in ws)} suns up")
    got = ctx.evaluate_batched(specs)
    st = ctx.batch_stats()
    _say(f"[batched] stats {st}")
    assert st["items"] == sum(int((w.sweep.sun_xyz[:, 2] > 0).sum()) for w in ws)
    for i, (w, sp, g) in enumerate(zip(ws, specs, got)):
        _same(g, _plain(ctx, sp), f"job {i} vs per-sun path")
        ref = oracle_lib.evaluate(w.scene, w.gen, w.sweep, w.map_n, w.k)
        assert np.array_equal(g.counts, ref.counts), f"job {i}: counts differ from the oracle"
        np.testing.assert_allclose(g.power, ref.power, rtol=1e-6, atol=0)
        np.testing.assert_allclose(g.energy, ref.energy, rtol=1e-6, atol=0)
    assert int(got[-1].counts[12].sum()) == 3200        # C1 winter noon, as the pinned oracle gives


def test_batched_full_raster_route_and_bin_limits(ctx):
    w = W.random_tiny(71, n_boxes=10, n_loose=50, n_mod_side=3, map_n=256, k=4, n_sun=6)
    base = _spec(ctx, w)
    ref = _plain(ctx, base)
    variants = [dict(full_raster=True), dict(bin_limit=1), dict(bin_limit=16, tile=32), dict(tile=32)]
    got = ctx.evaluate_batched([dict(base, **v) for v in variants])
    for v, g in zip(variants, got):
        _same(g, ref, f"variant {v}")


def test_batched_device_outputs_without_counts(ctx):
    import torch
    ws = _uneven_jobs()[:3]
    specs = [_spec(ctx, w) for w in ws]
    host = ctx.evaluate_batched(specs)
    dev = ctx.evaluate_batched([dict(sp, counts=False) for sp in specs], device=True)
    torch.cuda.synchronize()
    for h, d in zip(host, dev):
        assert d.counts is None
        assert np.array_equal(d.power.cpu().numpy(), h.power)
        assert np.array_equal(d.energy.cpu().numpy(), h.energy)


def test_slot_capacity_overflow_goes_to_per_sun_path(ctx):
    """With room for 2 records per slot nearly every sun overflows and is evaluated again by
    the per-sun path after the launch; results are unchanged."""
    ws = _uneven_jobs()[:4]
    specs = [_spec(ctx, w) for w in ws]
    ref = ctx.evaluate_batched(specs)
    try:
        ctx.batch_limits(max_slots=3, slot_records=2)
        got = ctx.evaluate_batched(specs)
        st = ctx.batch_stats()
    finally:
        ctx.batch_limits()
    _say(f"[batched] overflow stats {st}")
    assert st["redone"] > 0 and st["slots"] <= 3
    for r, g in zip(ref, got):
        _same(g, r, "capacity-limited batch")


def test_few_slots_many_items(ctx):
    """One slot: every item passes through the same work buffers in turn."""
    ws = _uneven_jobs()
    specs = [_spec(ctx, w) for w in ws]
    ref = ctx.evaluate_batched(specs)
    try:
        ctx.batch_limits(max_slots=1)
        got = ctx.evaluate_batched(specs)
        assert ctx.batch_stats()["slots"] == 1
    finally:
        ctx.batch_limits()
    for r, g in zip(ref, got):
        _same(g, r, "one-slot batch")


def test_xcd_placement_does_not_change_results(ctx):
    """Slots served by one XCD each (L1-only acquire) and by every XCD (full acquire)."""
    ws = _uneven_jobs()
    specs = [_spec(ctx, w) for w in ws]
    a = ctx.evaluate_batched(specs)
    ga = ctx.batch_stats()["xcd_groups"]
    try:
        ctx.batch_limits(any_xcd=True)
        b = ctx.evaluate_batched(specs)
        assert ctx.batch_stats()["xcd_groups"] == 1
    finally:
        ctx.batch_limits()
    _say(f"[batched] default placement: {ga} XCD groups")
    for x, y in zip(a, b):
        _same(x, y, "XCD placement")


def test_autotune_picks_a_candidate_with_identical_results(ctx):
    w = W.random_tiny(72, n_boxes=10, n_loose=40, n_mod_side=3, map_n=300, k=4, n_sun=8)
    sp = _spec(ctx, w)
    tile, lim, ms = ctx.autotune(sp, n_probe=4)
    _say(f"[autotune] tile={tile} bin_limit={lim} probe={ms:.3f} ms")
    assert tile in (32, 64) and lim in (8, 16, 32, 64, 128, 256) and ms > 0
    a = ctx.evaluate_batched([dict(sp, tile=tile, bin_limit=lim)])[0]
    _same(a, _plain(ctx, sp), "autotuned batch")


def test_autotune_cache_by_job_class(ctx, tmp_path):
    """A job of a class already tuned takes the cached choice without a launch; the cache
    survives a save and a load into another context; a cleared cache times again; a missing
    or malformed file is refused."""
    import json
    from paper_1410_5780_amd import pv3d
    ctx.tuning_cache(pv3d.TUNE_CLEAR)
    w1 = W.random_tiny(73, n_boxes=10, n_loose=40, n_mod_side=3, map_n=320, k=4, n_sun=8)
    w2 = W.random_tiny(74, n_boxes=9, n_loose=45, n_mod_side=3, map_n=320, k=4, n_sun=6)   # same class
    s1, s2 = _spec(ctx, w1), _spec(ctx, w2)
    first = ctx.autotune(s1, n_probe=4)
    stats = ctx.batch_stats()
    second = ctx.autotune(s2, n_probe=4)
    assert second == first and ctx.batch_stats() == stats      # cached: no launch
    path = str(tmp_path / "tuning.json")
    ctx.tuning_cache(pv3d.TUNE_SAVE, path)
    saved = json.load(open(path))
    assert len(saved) == 1 and saved[0]["map_n"] == 320 and saved[0]["k"] == 4
    assert (saved[0]["tile"], saved[0]["bin_limit"]) == first[:2]
    with pv3d.Context(0) as other:
        o2 = _spec(other, w2)
        other.tuning_cache(pv3d.TUNE_LOAD, path)
        assert other.autotune(o2, n_probe=4) == first
        assert other.batch_stats()["launch_us"] == 0                   # never launched
        other.tuning_cache(pv3d.TUNE_CLEAR)
        tile, lim, ms = other.autotune(o2, n_probe=4)
        assert other.batch_stats()["launch_us"] > 0 and tile in (32, 64)
    with pytest.raises(pv3d.Pv3dError) as e:
        ctx.tuning_cache(pv3d.TUNE_LOAD, str(tmp_path / "missing.json"))
    assert e.value.code == pv3d.ENOENT
    bad = tmp_path / "bad.json"
    bad.write_text(json.dumps([dict(saved[0], tile=128)]))
    with pytest.raises(pv3d.Pv3dError) as e:
        ctx.tuning_cache(pv3d.TUNE_LOAD, str(bad))
    assert e.value.code == pv3d.EINVAL
    bad.write_text('[{"map_n": 320}]')
    with pytest.raises(pv3d.Pv3dError) as e:
        ctx.tuning_cache(pv3d.TUNE_LOAD, str(bad))
    assert e.value.code == pv3d.EINVAL
    with pytest.raises(pv3d.Pv3dError) as e:
        ctx.tuning_cache(7)
    assert e.value.code == pv3d.EINVAL


def test_batched_argument_errors(ctx):
    from paper_1410_5780_amd import pv3d
    w = W.c1_tiny()
    sp = _spec(ctx, w)
    with pytest.raises(pv3d.Pv3dError) as e:
        ctx.evaluate_batched([dict(sp, tile=128)])
    assert e.value.code == pv3d.EINVAL
    with pytest.raises(pv3d.Pv3dError) as e:
        ctx.evaluate_batched([dict(sp, bin_limit=300)])
    assert e.value.code == pv3d.EINVAL
    with pytest.raises(pv3d.Pv3dError) as e:
        ctx.evaluate_batched([sp, dict(sp, scene=sp["scene"] + 999)])
    assert e.value.code == pv3d.ENOENT
    assert ctx.evaluate_batched([]) == []


def test_all_suns_below_horizon(ctx):
    w = W.c1_tiny()
    night = w.sweep.subset([0, 1, 2, 22, 23])
    sp = _spec(ctx, W.Workload("night", w.scene, w.gen, night, w.map_n, w.k))
    g = ctx.evaluate_batched([sp])[0]
    assert g.counts.sum() == 0 and np.all(g.power == 0) and np.all(g.energy == 0)


def test_c2_row_plant_sampled_suns_batched(ctx, oracle_lib):
    yr = W.year_sweep()
    idx = [0, 100, 1500, 2200, 3000, 4378]
    w = W.c2_row_plant(sweep=yr.subset(idx))
    sp = _spec(ctx, w)
    _say(f"[batched] C2 {w.scene.n_tri} tris, {len(idx)} suns")
    g = ctx.evaluate_batched([sp])[0]
    ref = oracle_lib.evaluate(w.scene, w.gen, w.sweep, w.map_n, w.k)
    assert np.array_equal(g.counts, ref.counts)
    np.testing.assert_allclose(g.power, ref.power, rtol=1e-6, atol=0)
    _same(g, _plain(ctx, sp), "C2 batched vs per-sun path")


def test_batched_at_the_largest_sizes(ctx, oracle_lib):
    """The ABI's largest sizes in one launch: N = 16384, and k = 255 with ideal strings and with the
    single-diode model. Every job equals the per-sun path, and its counts equal the oracle's."""
    import dataclasses
    big = W.random_tiny(81, n_boxes=6, n_loose=40, n_mod_side=3, map_n=16384, k=8, n_sun=2)
    dense = W.random_tiny(81, n_boxes=6, n_loose=6, n_mod_side=2, map_n=256, k=255, n_sun=2)
    diode = dataclasses.replace(dense, gen=dataclasses.replace(dense.gen, diode=W.DIODE_CELL), name="tiny81_diode")
    ws = [big, dense, diode]
    specs = [_spec(ctx, w) for w in ws]
    got = ctx.evaluate_batched(specs)
    for w, sp, g in zip(ws, specs, got):
        # the per-sun path at its own tile size (128 texels at N = 16384): results do not depend on it
        alone = ctx.evaluate(sp["scene"], sp["gen"], sp["generator"], sp["sweep"], sp["map_n"], sp["k"])
        _same(g, alone, f"{w.name} N={w.map_n} k={w.k}")
        ref = oracle_lib.evaluate(w.scene, w.gen, w.sweep, w.map_n, w.k)
        assert np.array_equal(np.asarray(g.counts), ref.counts), w.name
        assert int(ref.counts.sum()) > 1000
    _say(f"[batched] largest sizes: identical to the per-sun path; stats {ctx.batch_stats()}")
