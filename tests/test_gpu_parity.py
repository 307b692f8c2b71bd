"""HIP path vs the CPU oracle, through the C ABI (needs an MI355X).

Depth pictures, shaded flags and per-cell counts must be bit-exact; powers and
energies within 1e-6 relative (the arithmetic is the same sequence of IEEE
operations on both sides, so they are expected to agree exactly).
"""
import math
import sys

import numpy as np
import pytest

from paper_1410_5780_amd import workloads as W
from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu

REL = 1e-6


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


def compare(ctx, oracle_lib, w, maps=True, bits=True, tile=0, threads=0):
    _say(f"[parity] {w.name}: tris={w.scene.n_tri} cells={w.gen.n_cells} suns={w.sweep.n} "
         f"N={w.map_n} k={w.k} tile={tile}")
    sh = ctx.load_scene(w.scene)
    gh = ctx.define_generator(w.gen)
    try:
        got = ctx.evaluate(sh, gh, w.gen, w.sweep, w.map_n, w.k, export_depth=maps, export_bits=bits, tile=tile)
    finally:
        ctx.release_scene(sh)
        ctx.release_generator(gh)
    sh = ctx.load_scene(w.scene)
    gh = ctx.define_generator(w.gen)
    try:                      # the production route: picture only at sample texels, nothing exported
        lean = ctx.evaluate(sh, gh, w.gen, w.sweep, w.map_n, w.k, tile=tile, export_bits=bits)
    finally:
        ctx.release_scene(sh)
        ctx.release_generator(gh)
    ref = oracle_lib.evaluate(w.scene, w.gen, w.sweep, w.map_n, w.k, export_maps=maps, export_bits=bits,
                              threads=threads)
    assert np.array_equal(lean.counts, ref.counts)
    if bits:
        assert np.array_equal(lean.bits, ref.bits)
    np.testing.assert_allclose(lean.power, ref.power, rtol=REL, atol=0)
    assert ref.outside == 0
    if maps:
        bad = np.nonzero((got.maps != ref.maps).reshape(w.sweep.n, -1).any(axis=1))[0]
        assert bad.size == 0, f"depth pictures differ at suns {bad[:10]}: " \
            f"{int((got.maps[bad[0]] != ref.maps[bad[0]]).sum())} texels"
    if bits:
        assert np.array_equal(got.bits, ref.bits)
    assert np.array_equal(got.counts, ref.counts)
    np.testing.assert_allclose(got.power, ref.power, rtol=REL, atol=0)
    np.testing.assert_allclose(got.power_ref, ref.power_ref, rtol=REL, atol=0)
    np.testing.assert_allclose(got.energy, ref.energy, rtol=REL, atol=0)
    exact = np.array_equal(got.power, ref.power) and np.array_equal(got.energy, ref.energy)
    _say(f"[parity] {w.name}: ok (powers bit-identical: {exact}); shaded={int(got.counts.sum())}")
    return got, ref


def test_c1_tiny_full(ctx, oracle_lib):
    for d in (0.0, 100.0):
        got, ref = compare(ctx, oracle_lib, W.c1_tiny(d_poa=d))
        assert int(got.counts[12].sum()) == 3200
    assert got.loss == pytest.approx(0.04670964, abs=5e-9)


@pytest.mark.parametrize("seed,n,k,tile", [(31, 200, 3, 64), (32, 130, 4, 32), (33, 257, 1, 128),
                                           (34, 64, 16, 0), (35, 16, 2, 64), (36, 333, 5, 32)])
def test_random_tiny_ragged(ctx, oracle_lib, seed, n, k, tile):
    w = W.random_tiny(seed, n_boxes=10, n_loose=40, n_mod_side=3, map_n=n, k=k, n_sun=8)
    compare(ctx, oracle_lib, w, tile=tile)


@pytest.mark.parametrize("seed,n", [(61, 256), (62, 200)])
def test_dense_tiles_split_in_quadrants(ctx, oracle_lib, seed, n):
    """Thousands of loose triangles over the generator: 64-texel tiles hold far
    more than the 128 bin entries above which the tile pass takes a tile as four
    quadrant items (a ragged map at n = 200)."""
    w = W.random_tiny(seed, n_boxes=4, n_loose=6000, n_mod_side=3, map_n=n, k=4, n_sun=5)
    compare(ctx, oracle_lib, w, tile=64)


def test_tile_sizes_give_identical_results(ctx):
    w = W.random_tiny(41, n_boxes=12, n_loose=60, n_mod_side=3, map_n=300, k=4, n_sun=5)
    sh, gh = ctx.load_scene(w.scene), ctx.define_generator(w.gen)
    outs = [ctx.evaluate(sh, gh, w.gen, w.sweep, w.map_n, w.k, export_depth=True, export_bits=True, tile=t)
            for t in (32, 64, 128)]
    for o in outs[1:]:
        assert np.array_equal(o.maps, outs[0].maps) and np.array_equal(o.bits, outs[0].bits)
        assert np.array_equal(o.power, outs[0].power)


@pytest.mark.parametrize("seed,n,k", [(42, 256, 4), (43, 190, 3)])
def test_separate_test_route_matches_fused_route(ctx, seed, n, k):
    """Depth check in a second kernel reading the materialised picture == check inside the tile."""
    w = W.random_tiny(seed, n_boxes=10, n_loose=50, n_mod_side=3, map_n=n, k=k, n_sun=6)
    sh, gh = ctx.load_scene(w.scene), ctx.define_generator(w.gen)
    a = ctx.evaluate(sh, gh, w.gen, w.sweep, w.map_n, w.k, export_depth=True, export_bits=True)
    b = ctx.evaluate(sh, gh, w.gen, w.sweep, w.map_n, w.k, export_depth=True, export_bits=True, separate_test=True)
    c = ctx.evaluate(sh, gh, w.gen, w.sweep, w.map_n, w.k, separate_test=True)
    d = ctx.evaluate(sh, gh, w.gen, w.sweep, w.map_n, w.k, export_bits=True)                    # sparse
    e = ctx.evaluate(sh, gh, w.gen, w.sweep, w.map_n, w.k, export_bits=True, full_raster=True)  # full, no export
    assert np.array_equal(a.maps, b.maps) and np.array_equal(a.bits, b.bits)
    assert np.array_equal(a.bits, d.bits) and np.array_equal(a.bits, e.bits)
    for o in (b, c, d, e):
        assert np.array_equal(a.counts, o.counts) and np.array_equal(a.power, o.power)


def test_empty_scene_and_backlit_and_below_horizon(ctx, oracle_lib):
    c1 = W.c1_tiny(d_poa=30.0)
    empty = W.Workload("empty_scene", W.Scene(np.zeros((0, 3)), np.zeros((0, 3), np.int32)), c1.gen,
                       W.make_sweep(40.4, [1, 172, 355], np.arange(0.0, 24.0, 1.0), d_poa=30.0), 256, 4)
    got, _ = compare(ctx, oracle_lib, empty)
    assert got.counts.sum() == 0
    # north-facing module at winter noon: back-lit above the horizon
    g = W.c1_tiny().gen
    g.edge_v = g.edge_v * np.array([[1.0, -1.0, 1.0]])
    g.edge_u = -g.edge_u
    back = W.Workload("backlit", c1.scene, g, W.make_sweep(40.4, [355], [10.0, 12.0, 14.0, 23.0], d_poa=30.0), 128, 3)
    got, _ = compare(ctx, oracle_lib, back)
    assert got.counts.sum() == 0 and np.all(got.maps == (1 << 24) - 1)


def _parallel_occluders(seed, n_sun=16, split=1):
    """Six tilted modules, each with two quads parallel to it over part of its face, offset along its
    normal by a few millimetres to a few centimetres either way and by a few micrometres (a depth unit
    here is about 1 um): the cases around the depth bias, where a triangle just in front of a module or
    the module's own triangles must not shade it and one farther in front must. With split > 1 every
    quad is cut into split x split smaller ones, so that a tile holds enough entries to go to the
    workgroup route."""
    rng = np.random.default_rng(seed)
    gen = W.module_rows(2, 3, tilt_deg=float(rng.uniform(10, 40)), pitch=3.0, z0=0.4, modules_per_string=3)
    n = np.cross(gen.edge_u, gen.edge_v)
    n /= np.linalg.norm(n, axis=1, keepdims=True)
    offs = np.concatenate([rng.uniform(-0.06, 0.06, 8), rng.choice([-1, 1], 4) * rng.uniform(1e-6, 2e-5, 4)])
    rng.shuffle(offs)
    quads = []
    for m in range(gen.n_mod):
        for q in range(2):
            a0, a1 = np.sort(rng.uniform(0.0, 1.0, 2))
            b0, b1 = np.sort(rng.uniform(0.0, 1.0, 2))
            o = gen.origin[m] + offs[2 * m + q] * n[m]
            u, v = gen.edge_u[m], gen.edge_v[m]
            ga, gb = np.linspace(a0, a1, split + 1), np.linspace(b0, b1, split + 1)
            for i in range(split):
                for j in range(split):
                    quads.append([o + ga[i] * u + gb[j] * v, o + ga[i + 1] * u + gb[j] * v,
                                  o + ga[i + 1] * u + gb[j + 1] * v, o + ga[i] * u + gb[j + 1] * v])
    mesh = W._Mesh()
    mesh.add(np.array(quads), np.array([[0, 1, 2], [0, 2, 3]]))
    days = rng.integers(1, 366, n_sun)
    hours = rng.uniform(6.5, 17.5, n_sun)
    s = W.cooper_sun(W.LAT_DEG, days, hours)
    sw = W.Sweep(np.ascontiguousarray(s), np.full(n_sun, 900.0), np.full(n_sun, 80.0), np.full(n_sun, 1.0),
                 days.astype(np.int32), hours)
    return W.Workload(f"parallel{seed}x{split}", mesh.scene(), gen, sw, 256, 4, "occluders parallel to the modules")


@pytest.mark.parametrize("seed", [11, 12, 13, 14])
def test_occluders_parallel_to_the_modules_near_the_bias(ctx, oracle_lib, seed):
    """The tile pass leaves out of a module's tests the triangles that lie far enough behind its plane
    (its own, one just in front within the bias, one behind it); the oracle tests every triangle."""
    got, _ = compare(ctx, oracle_lib, _parallel_occluders(seed), maps=False, bits=True)
    assert got.counts.sum() > 0


@pytest.mark.parametrize("seed", [21, 22])
def test_dense_occluders_parallel_to_the_modules_near_the_bias(ctx, oracle_lib, seed):
    """The same occluders cut into 64 quads each (up to about 256 bin entries per tile): the
    workgroup route's early return, which drops a tile when every triangle reaching it lies behind
    the plane of every module there, against the oracle."""
    got, _ = compare(ctx, oracle_lib, _parallel_occluders(seed, split=8), maps=False, bits=True)
    assert got.counts.sum() > 0


def test_guard_band_clip_path(ctx, oracle_lib):
    """A vertical module seen almost edge-on makes the window very thin, so scene geometry a
    few metres away lies millions of texels out and goes through the guard-band clip."""
    gen = W.Generator(np.array([[0.0, 0.0, 0.5]]), np.array([[0.936, 0.0, 0.0]]), np.array([[0.0, 0.0, 1.56]]),
                      6, 10, W.portrait_substrings(), 3, np.zeros(1, np.int32))
    assert np.allclose(np.cross(gen.edge_u[0], gen.edge_v[0]) / 1.46016, [0, -1, 0])
    s = np.array([[1.0, -0.001, 0.05], [1.0, -0.002, 0.3], [0.6, -0.8, 0.2]])
    s /= np.linalg.norm(s, axis=1, keepdims=True)
    sw = W.Sweep(s, np.full(3, 1000.0), np.full(3, 20.0), np.ones(3), np.zeros(3, np.int32), np.zeros(3))
    m = W._Mesh()
    m.add(*W.ground_plane(-100, -100, 100, 100, 0.0))
    m.add(*W.boxes(0.5, -3.0, 0.2, 0.2, 0.0, 4.0, 0.0))
    m.add(*W.boxes(-2.0, -1.0, 0.5, 0.5, 0.0, 2.0, 0.3))
    w = W.Workload("clip", m.scene(), gen, sw, 512, 4)
    compare(ctx, oracle_lib, w)


def test_device_outputs_match_host_outputs(ctx):
    import torch
    w = W.random_tiny(51, n_boxes=8, n_loose=30, n_mod_side=3, map_n=192, k=4, n_sun=6)
    sh, gh = ctx.load_scene(w.scene), ctx.define_generator(w.gen)
    host = ctx.evaluate(sh, gh, w.gen, w.sweep, w.map_n, w.k)
    counts = torch.zeros((w.sweep.n, w.gen.n_cells), dtype=torch.int32, device="cuda")
    dev = ctx.evaluate_device(sh, gh, w.gen, w.sweep, w.map_n, w.k, counts=counts)
    torch.cuda.synchronize()
    assert np.array_equal(counts.cpu().numpy().view(np.uint32), host.counts)
    assert np.array_equal(dev.power.cpu().numpy(), host.power)
    assert np.array_equal(dev.energy.cpu().numpy(), host.energy)


def test_device_outputs_on_torch_default_stream_are_ordered_with_it(ctx):
    """Device outputs of a call made on torch's default (null) stream are read by torch right
    away, with no device-wide synchronization: the reads must come after the library's writes."""
    import torch
    w = W.random_tiny(52, n_boxes=10, n_loose=300, n_mod_side=4, map_n=768, k=6, n_sun=48)
    sh, gh = ctx.load_scene(w.scene), ctx.define_generator(w.gen)
    host = ctx.evaluate(sh, gh, w.gen, w.sweep, w.map_n, w.k)
    assert torch.cuda.current_stream().cuda_stream == 0
    for _ in range(3):
        counts = torch.full((w.sweep.n, w.gen.n_cells), -1, dtype=torch.int32, device="cuda")
        dev = ctx.evaluate_device(sh, gh, w.gen, w.sweep, w.map_n, w.k, counts=counts)
        got_energy = dev.energy.cpu().numpy()          # ordered on torch's stream only
        got_counts = counts.cpu().numpy().view(np.uint32)
        assert np.array_equal(got_energy, host.energy)
        assert np.array_equal(got_counts, host.counts)
    ctx.release_scene(sh)
    ctx.release_generator(gh)


def test_path_stats_count_the_last_evaluation():
    """Zero before any evaluation; after one, the suns and the set-up records of the up suns:
    at least one record per triangle the window keeps, at most five (a clipped triangle's fan)."""
    from paper_1410_5780_amd import pv3d
    w = W.c1_tiny(d_poa=100.0)
    with pv3d.Context(0) as c:
        assert c.path_stats() == {"suns": 0, "records": 0, "large": 0, "pairs": 0}
        sh, gh = c.load_scene(w.scene), c.define_generator(w.gen)
        c.evaluate(sh, gh, w.gen, w.sweep, w.map_n, w.k)
        st = c.path_stats()
    n_up = int((w.sweep.sun_xyz[:, 2] > 0).sum())
    tris = w.scene.n_tri + 2 * w.gen.n_mod
    assert st["suns"] == w.sweep.n and 0 < st["records"] <= 5 * tris * n_up and st["pairs"] > 0


def test_argument_errors(ctx):
    from paper_1410_5780_amd import pv3d
    w = W.c1_tiny()
    sh, gh = ctx.load_scene(w.scene), ctx.define_generator(w.gen)
    with pytest.raises(pv3d.Pv3dError) as e:
        ctx.evaluate(sh, gh, w.gen, w.sweep, 8, 4)
    assert e.value.code == pv3d.EINVAL
    with pytest.raises(pv3d.Pv3dError) as e:
        ctx.evaluate(sh, gh, w.gen, w.sweep, 64, 0)
    assert e.value.code == pv3d.EINVAL
    bad = w.sweep.subset([12])
    bad.sun_xyz = bad.sun_xyz * 1.01
    with pytest.raises(pv3d.Pv3dError) as e:
        ctx.evaluate(sh, gh, w.gen, bad, 64, 2)
    assert e.value.code == pv3d.EINVAL
    with pytest.raises(pv3d.Pv3dError) as e:
        ctx.evaluate(sh + 1000, gh, w.gen, w.sweep, 64, 2)
    assert e.value.code == pv3d.ENOENT
    nan = W.Scene(np.array([[0.0, 0.0, np.nan], [1, 0, 0], [0, 1, 0]]), np.array([[0, 1, 2]], np.int32))
    with pytest.raises(pv3d.Pv3dError) as e:
        ctx.load_scene(nan)
    assert e.value.code == pv3d.EINVAL
    small = pv3d.Context(0, budget_bytes=1 << 20)
    with pytest.raises(pv3d.Pv3dError) as e:
        small.load_scene(W.c2_row_plant(sweep=w.sweep.subset([12])).scene)
    assert e.value.code == pv3d.ENOMEM
    small.close()


# ---------------------------------------------------------------------------
# full-size configurations on sampled suns
# ---------------------------------------------------------------------------
def test_c2_row_plant_full_size_sampled_suns(ctx, oracle_lib):
    yr = W.year_sweep()
    idx = [0, 100, 1500, 2200, 3000, 4378]          # low winter, morning, spring, summer dusk, afternoon, last
    w = W.c2_row_plant(sweep=yr.subset(idx))
    got, ref = compare(ctx, oracle_lib, w)
    assert got.counts.sum() > 0


def test_c3_rooftop_full_size_sampled_suns(ctx, oracle_lib):
    yr = W.year_sweep()
    w = W.c3_rooftop(sweep=yr.subset([700, 2200]))
    got, ref = compare(ctx, oracle_lib, w, bits=False)
    assert got.counts.sum() > 0


@pytest.mark.parametrize("which", ["c3", "c2"])
def test_full_size_production_route_on_24_suns(ctx, oracle_lib, which):
    """The production route (nothing exported but the shaded flags) on every 183rd sun of the
    year at full size: two groups of twelve suns, one on each lane, against the oracle."""
    yr = W.year_sweep()
    sub = yr.subset(np.arange(0, yr.n, 183))
    w = W.c3_rooftop(sweep=sub) if which == "c3" else W.c2_row_plant(sweep=sub)
    _say(f"[parity] {w.name} production route: {sub.n} suns")
    sh, gh = ctx.load_scene(w.scene), ctx.define_generator(w.gen)
    try:
        got = ctx.evaluate(sh, gh, w.gen, w.sweep, w.map_n, w.k, export_bits=True)
    finally:
        ctx.release_scene(sh)
        ctx.release_generator(gh)
    ref = oracle_lib.evaluate(w.scene, w.gen, w.sweep, w.map_n, w.k, export_bits=True)
    bad = np.nonzero((got.counts != ref.counts).any(axis=1))[0]
    assert bad.size == 0, f"counts differ at suns {bad[:10]}"
    assert np.array_equal(got.bits, ref.bits)
    np.testing.assert_allclose(got.power, ref.power, rtol=REL, atol=0)
    np.testing.assert_allclose(got.power_ref, ref.power_ref, rtol=REL, atol=0)
    np.testing.assert_allclose(got.energy, ref.energy, rtol=REL, atol=0)
    assert ref.outside == 0 and got.counts.sum() > 0


def test_back_to_back_device_evaluations_on_two_streams(ctx, oracle_lib):
    """Two asynchronous evaluations queued at once on two streams share the context's work
    buffers: the second waits for the first, and both equal the oracle."""
    import torch
    ws = [W.random_tiny(61, n_sun=7, map_n=160, k=3), W.random_tiny(62, n_boxes=9, n_sun=5, map_n=224, k=4)]
    hs = [(ctx.load_scene(w.scene), ctx.define_generator(w.gen)) for w in ws]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    _say("[parity] two device evaluations on two streams")
    counts = [torch.zeros((w.sweep.n, w.gen.n_cells), dtype=torch.int32, device="cuda") for w in ws]
    torch.cuda.synchronize()
    got = [ctx.evaluate_device(sh, gh, w.gen, w.sweep, w.map_n, w.k, stream=st, counts=c)
           for (sh, gh), w, st, c in zip(hs, ws, streams, counts)]
    torch.cuda.synchronize()
    for w, g, c, (sh, gh) in zip(ws, got, counts, hs):
        ref = oracle_lib.evaluate(w.scene, w.gen, w.sweep, w.map_n, w.k)
        assert np.array_equal(c.cpu().numpy().view(np.uint32), ref.counts), w.name
        np.testing.assert_allclose(g.power.cpu().numpy(), ref.power, rtol=REL, atol=0)
        np.testing.assert_allclose(g.energy.cpu().numpy(), ref.energy, rtol=REL, atol=0)
        ctx.release_scene(sh)
        ctx.release_generator(gh)
