"""Serving loop: jobs submitted while others run share one live persistent
launch. Each job's result must be the same, bit for bit, alone (the per-sun
path) and in the mix, and must match the CPU oracle: counts equal, powers and
energies within 1e-6 relative (needs an MI355X)."""
import sys
import time

import numpy as np
import pytest

from paper_1410_5780_amd import workloads as W
from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture()
def ctx():
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_1410_5780_amd import pv3d
    c = pv3d.Context(0)
    yield c
    c.close()


def _spec(ctx, w, **kw):
    d = dict(scene=ctx.load_scene(w.scene), gen=ctx.define_generator(w.gen), generator=w.gen, sweep=w.sweep,
             map_n=w.map_n, k=w.k)
    d.update(kw)
    return d


def _alone(ctx, sp):
    return ctx.evaluate(sp["scene"], sp["gen"], sp["generator"], sp["sweep"], sp["map_n"], sp["k"],
                        tile=sp.get("tile", 0) or 64)


def _same(a, b, what):
    ca, cb = np.asarray(a.counts), np.asarray(b.counts)
    if not np.array_equal(ca, cb):
        bad = np.argwhere(ca != cb)
        raise AssertionError(f"{what}: counts differ at {len(bad)} cells, first {bad[:5].tolist()}, "
                             f"got {ca[tuple(bad[0])]} want {cb[tuple(bad[0])]}")
    assert np.array_equal(np.asarray(a.power), np.asarray(b.power)), f"{what}: power differs"
    assert np.array_equal(np.asarray(a.power_ref), np.asarray(b.power_ref)), f"{what}: power_ref differs"
    assert np.array_equal(np.asarray(a.energy), np.asarray(b.energy)), f"{what}: energy differs"


def _oracle_same(got, w, oracle_lib, what, ref=None):
    """Served result against the oracle on the same inputs: counts bit-exact, powers and
    energy within 1e-6 relative (they are in fact identical)."""
    if ref is None:
        ref = oracle_lib.evaluate(w.scene, w.gen, w.sweep, w.map_n, w.k)
    c = np.asarray(got.counts.cpu().numpy().view(np.uint32) if hasattr(got.counts, "cpu") else got.counts)
    if not np.array_equal(c, ref.counts):
        bad = np.argwhere(c != ref.counts)
        raise AssertionError(f"{what}: counts differ from the oracle at {len(bad)} cells, first {bad[:5].tolist()}")
    for name in ("power", "power_ref", "energy"):
        a = getattr(got, name)
        a = a.cpu().numpy() if hasattr(a, "cpu") else np.asarray(a)
        assert np.allclose(a, getattr(ref, name), rtol=1e-6, atol=0), f"{what}: {name} differs from the oracle"


def _mix():
    ws = [W.random_tiny(80 + i, n_boxes=6 + i, n_loose=20 + 5 * i, n_mod_side=2 + i % 2, map_n=128 + 40 * i,
                        k=2 + i % 3, n_sun=5 + i) for i in range(6)]
    ws.append(W.c1_tiny(d_poa=100.0))
    yr = W.year_sweep()
    ws.append(W.c2_row_plant(sweep=yr.subset(list(range(1000, 1200, 10)))))     # 20 suns of the big plant
    return ws


def test_results_same_alone_and_in_the_mix(ctx, oracle_lib):
    ws = _mix()
    specs = [_spec(ctx, w, tile=(32 if i % 3 == 1 else 0)) for i, w in enumerate(ws)]
    _say(f"[serve] {len(specs)} jobs submitted together")
    tickets = [ctx.submit(sp) for sp in specs]
    got = [ctx.wait(t) for t in tickets]
    for i, (w, sp, g) in enumerate(zip(ws, specs, got)):
        _oracle_same(g, w, oracle_lib, f"job {i} ({w.name})")
        _same(g, _alone(ctx, sp), f"job {i}")
    st = ctx.serve_stats()
    _say(f"[serve] stats {st}")
    assert st["jobs_done"] == len(specs)
    assert int(got[6].counts[12].sum()) == 3200          # C1 winter noon


def test_jobs_arriving_while_others_run_share_the_launch(ctx):
    """Staggered arrivals: later jobs join the launch that already runs the first ones."""
    yr = W.year_sweep()
    big = W.c2_row_plant(sweep=yr.subset(list(range(0, yr.n, 60))))              # 73 suns, tens of ms
    bs = _spec(ctx, big)
    small = [_spec(ctx, w) for w in _mix()[:6]]
    t0 = ctx.submit(bs)
    tickets = []
    for sp in small:
        time.sleep(0.002)
        tickets.append(ctx.submit(sp))
    g0 = ctx.wait(t0)
    got = [ctx.wait(t) for t in tickets]
    st = ctx.serve_stats()
    _say(f"[serve] staggered stats {st}")
    assert st["launches"] < 1 + len(small)               # arrivals joined a running launch
    _same(g0, _alone(ctx, bs), "big job")
    for i, (sp, g) in enumerate(zip(small, got)):
        _same(g, _alone(ctx, sp), f"small job {i}")


def test_scene_in_use_cannot_be_released(ctx):
    from paper_1410_5780_amd import pv3d
    yr = W.year_sweep()
    sp = _spec(ctx, W.c2_row_plant(sweep=yr.subset(list(range(0, yr.n, 50)))))
    t = ctx.submit(sp)
    with pytest.raises(pv3d.Pv3dError) as e:
        ctx.release_scene(sp["scene"])
    assert e.value.code == pv3d.EBUSY
    ctx.wait(t)
    ctx.release_scene(sp["scene"])


@pytest.fixture()
def small_ctx():
    """64 MB of budget and small slots: the job arena holds about four year-long tiny jobs."""
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_1410_5780_amd import pv3d
    c = pv3d.Context(0, budget_bytes=64 << 20)
    c.batch_limits(slot_records=4096)
    yield c
    c.close()


def _tiny_year(c, seed=90, every=2):
    yr = W.year_sweep()
    w = W.random_tiny(seed, n_boxes=8, n_loose=20, n_mod_side=3, map_n=256, k=4, n_sun=4)
    w = W.Workload("tiny_year", w.scene, w.gen, yr.subset(list(range(0, yr.n, every))), 256, 4)
    return w, _spec(c, w)


def _oracle_ref(w, oracle_lib):
    return oracle_lib.evaluate(w.scene, w.gen, w.sweep, w.map_n, w.k)


def test_admission_by_hbm_budget(small_ctx, oracle_lib):
    """Jobs that fit the arena a few at a time wait for memory and all complete with the
    oracle's results; a job that can never fit is refused with ENOMEM."""
    from paper_1410_5780_amd import pv3d
    c = small_ctx
    w, sp = _tiny_year(c)
    ref = _oracle_ref(w, oracle_lib)
    tickets = [c.submit(sp) for _ in range(6)]
    got = [c.wait(t) for t in tickets]
    for g in got:
        _oracle_same(g, w, oracle_lib, "budget-limited job", ref)
    yr = W.year_sweep()
    many = W.Sweep(*(np.tile(a, (200,) + (1,) * (a.ndim - 1)) for a in (yr.sun_xyz, yr.dni, yr.d_poa, yr.dt_h,
                                                                          yr.day, yr.hour)))
    with pytest.raises(pv3d.Pv3dError) as e:
        c.submit(dict(sp, sweep=many))
    assert e.value.code == pv3d.ENOMEM
    _say(f"[serve] budget stats {c.serve_stats()}")


def test_cancel(small_ctx, oracle_lib):
    """A job waiting for memory is cancelled before it runs; the others are unaffected."""
    from paper_1410_5780_amd import pv3d
    c = small_ctx
    w, sp = _tiny_year(c, every=1)                       # about 9.5 MB of counts: two fill the arena
    ref = _oracle_ref(w, oracle_lib)
    ta, tb, tc, td = (c.submit(sp) for _ in range(4))
    c.cancel(td)                                          # still waiting for memory
    ra = c.wait(ta)
    with pytest.raises(pv3d.Pv3dError) as e:
        c.wait(td)
    assert e.value.code == pv3d.ECANCELED
    for t in (tb, tc):
        _oracle_same(c.wait(t), w, oracle_lib, "job next to a cancelled one", ref)
    _oracle_same(ra, w, oracle_lib, "first job", ref)
    with pytest.raises(pv3d.Pv3dError) as e:
        c.wait(td)                                        # forgotten
    assert e.value.code == pv3d.ENOENT


def test_device_outputs(ctx, oracle_lib):
    import torch
    ws = _mix()[:4]
    specs = [_spec(ctx, w) for w in ws]
    tickets = [ctx.submit(sp, device=True) for sp in specs]
    got = [ctx.wait(t) for t in tickets]
    torch.cuda.synchronize()
    for w, sp, g in zip(ws, specs, got):
        _oracle_same(g, w, oracle_lib, f"device outputs of {w.name}")
        a = _alone(ctx, sp)
        assert np.array_equal(g.counts.cpu().numpy().view(np.uint32), a.counts)
        assert np.array_equal(g.power.cpu().numpy(), a.power)
        assert np.array_equal(g.energy.cpu().numpy(), a.energy)


def test_serving_after_the_per_sun_path_in_the_same_context(ctx):
    """A context that has run the per-sun path on its lanes, then starts its serving loop:
    every request of a burst of the configured stream completes, and the per-sun path
    still gives the same results with the loop running."""
    from paper_1410_5780_amd import serve
    yr = W.year_sweep()
    w = W.c2_row_plant(sweep=yr.subset(np.arange(0, yr.n, 10)))
    sh, gh = ctx.load_scene(w.scene), ctx.define_generator(w.gen)
    first = ctx.evaluate(sh, gh, w.gen, w.sweep, w.map_n, w.k)
    reqs = W.serving_stream(seed=5, rate_hz=200.0, duration_s=0.1)
    t0 = time.perf_counter()
    res = serve.run_stream(ctx, reqs, seed=5, log=_say)
    wall = time.perf_counter() - t0
    _say(f"[serve] after the per-sun path: {res['requests']} requests in {wall:.2f} s, p99 {res['p99_ms']:.0f} ms")
    assert res["requests"] == len(reqs)
    assert res["p99_ms"] < 120000.0, "a request waited more than 2 minutes"
    again = ctx.evaluate(sh, gh, w.gen, w.sweep, w.map_n, w.k)
    _same(again, first, "per-sun path with the serving loop started")


def test_scene_loads_while_a_launch_is_live(ctx, oracle_lib):
    """Loading a scene and defining a generator while the loop serves a long job return without
    waiting for the live launch (their copies go on the context's own stream): the job is still
    running when they return, and both the job and a job on the new scene come out right."""
    big = W.c2_row_plant()                         # a year of the row plant: a few tenths of a second
    sp = _spec(ctx, big)
    t = ctx.submit(sp)
    small = W.random_tiny(97, n_boxes=6, n_loose=30, n_mod_side=2, map_n=160, k=3, n_sun=4)
    sp2 = _spec(ctx, small)                        # load_scene and define_generator during the job
    assert not ctx.poll(t), "the loads waited for the live launch"
    got = ctx.wait(t)
    _same(got, _alone(ctx, sp), "served while scenes were loaded")
    _oracle_same(ctx.wait(ctx.submit(sp2)), small, oracle_lib, "job on the scene loaded mid-run")


def test_suns_beyond_slot_capacity_are_evaluated_again(ctx, oracle_lib):
    """Slots of 64 records: the suns of a scene with hundreds of loose triangles overflow them,
    and the host evaluates just those suns again on the per-sun path. Every served result
    equals the per-sun path's, next to a job whose suns fit."""
    ctx.batch_limits(slot_records=64)
    ws = [W.random_tiny(95, n_boxes=6, n_loose=400, n_mod_side=3, map_n=192, k=4, n_sun=8), W.c1_tiny(d_poa=100.0)]
    specs = [_spec(ctx, w) for w in ws]
    served = [ctx.wait(t) for t in [ctx.submit(sp) for sp in specs]]
    for w, sp, got in zip(ws, specs, served):
        _same(got, _alone(ctx, sp), f"{w.name} served with slots of 64 records")
        _oracle_same(got, w, oracle_lib, f"{w.name} served with slots of 64 records")
    _say(f"[serve] overflow stats {ctx.serve_stats()}")
