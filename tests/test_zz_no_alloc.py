"""pv3d_evaluate_noalloc (work memory from the library's static device array,
nothing allocated by the call) against pv3d_evaluate on the same inputs:
identical counts, powers and energy, on two calls in a row (the second with a
smaller input), for a tracked generator, and for a scene that fits only with a
smaller bin_limit; a scene that does not fit is refused before anything runs."""
import sys

import numpy as np
import pytest

from tests.conftest import gpu_available
from paper_1410_5780_amd import workloads as W

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


def _outputs(w, with_counts=True):
    import torch
    n = w.sweep.n
    counts = torch.full((n, w.gen.n_cells), -1, dtype=torch.int32, device="cuda") if with_counts else None
    return (counts, torch.full((n,), np.nan, dtype=torch.float64, device="cuda"),
            torch.full((n,), np.nan, dtype=torch.float64, device="cuda"),
            torch.full((2,), np.nan, dtype=torch.float64, device="cuda"))


def _check_same(ctx, w, bin_limit=0, tile=0, with_counts=True):
    """pv3d_evaluate (the context's own work buffers) and pv3d_evaluate_noalloc, bit for bit."""
    import torch
    sh, gh = ctx.load_scene(w.scene), ctx.define_generator(w.gen)
    try:
        _say(f"[noalloc] {w.name}: {w.sweep.n} suns, N={w.map_n}, k={w.k}, bin_limit={bin_limit}, tile={tile}")
        ref_counts = torch.zeros((w.sweep.n, w.gen.n_cells), dtype=torch.int32, device="cuda")
        ref = ctx.evaluate_device(sh, gh, w.gen, w.sweep, w.map_n, w.k, counts=ref_counts, tile=tile)
        c, pw, pr, en = _outputs(w, with_counts)
        got = ctx.evaluate_noalloc(sh, gh, w.gen, w.sweep, w.map_n, w.k, c, pw, pr, en, tile=tile,
                                   bin_limit=bin_limit)
        torch.cuda.synchronize()
        if with_counts:
            assert torch.equal(got.counts, ref_counts), f"{w.name}: counts differ"
        for name in ("power", "power_ref", "energy"):
            a, b = getattr(got, name).cpu().numpy(), getattr(ref, name).cpu().numpy()
            assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), f"{w.name}: {name} differs"
        assert (ref_counts.sum().item() > 0) == (ref.loss > 0)
    finally:
        ctx.release_scene(sh)
        ctx.release_generator(gh)


def test_two_calls_in_a_row_the_second_smaller(ctx):
    """A call with many suns (groups of suns on two lanes) and then a smaller one, which finds
    the first call's contents in the array."""
    big = W.random_tiny(71, n_boxes=12, n_loose=400, n_mod_side=4, map_n=512, k=4, n_sun=40)
    small = W.random_tiny(72, n_boxes=5, n_loose=30, n_mod_side=2, map_n=200, k=3, n_sun=5)
    _check_same(ctx, big)
    _check_same(ctx, small)


def test_without_counts_and_with_other_tiles(ctx):
    w = W.random_tiny(73, n_boxes=8, n_loose=60, n_mod_side=3, map_n=300, k=5, n_sun=9)
    _check_same(ctx, w, with_counts=False)
    _check_same(ctx, w, tile=32)


def test_tracked_generator(ctx):
    _check_same(ctx, W.tracker_pair(kind=2))


def test_scene_too_large_is_refused_and_fits_with_a_smaller_bin_limit(ctx):
    """40,000 loose triangles need about 200 MB of bins at the default bin_limit (256), more
    than the 128 MiB array: ERANGE before anything is queued. With bin_limit 8 the call fits,
    and its results equal pv3d_evaluate's at the default bin_limit."""
    import torch
    from paper_1410_5780_amd import pv3d
    w = W.random_tiny(74, n_boxes=6, n_loose=40000, n_mod_side=3, map_n=1024, k=4, n_sun=6)
    sh, gh = ctx.load_scene(w.scene), ctx.define_generator(w.gen)
    try:
        c, pw, pr, en = _outputs(w)
        _say("[noalloc] oversized scene: expect ERANGE")
        with pytest.raises(pv3d.Pv3dError) as ei:
            ctx.evaluate_noalloc(sh, gh, w.gen, w.sweep, w.map_n, w.k, c, pw, pr, en)
        assert ei.value.code == pv3d.ERANGE and "static scratch" in str(ei.value)
        torch.cuda.synchronize()
        assert bool(torch.isnan(pw).all()) and int(c.min().item()) == -1   # nothing was written
    finally:
        ctx.release_scene(sh)
        ctx.release_generator(gh)
    _check_same(ctx, w, bin_limit=8)


def test_dark_sweep_and_mixed_sweep(ctx):
    """Every sun below the horizon (nothing is drawn, every power zero), then a sweep whose up
    suns are split by night hours (groups skip the down suns in between)."""
    import dataclasses
    base = W.random_tiny(76, n_boxes=8, n_loose=50, n_mod_side=3, map_n=256, k=4, n_sun=2)
    night = W.make_sweep(40.4, [10, 200], [0.0, 1.0, 2.0, 22.0, 23.0])
    assert (night.sun_xyz[:, 2] <= 0.0).all()
    _check_same(ctx, dataclasses.replace(base, sweep=night, name="night"))
    mixed = W.make_sweep(40.4, [30, 172, 300], np.arange(0.0, 24.0, 1.0))
    assert (mixed.sun_xyz[:, 2] > 0.0).any() and (mixed.sun_xyz[:, 2] <= 0.0).any()
    _check_same(ctx, dataclasses.replace(base, sweep=mixed, name="day and night"))


def test_host_outputs_are_refused(ctx):
    from paper_1410_5780_amd import pv3d
    import ctypes
    w = W.random_tiny(75, n_sun=2)
    sh, gh = ctx.load_scene(w.scene), ctx.define_generator(w.gen)
    try:
        pw, pr, en = np.zeros(2), np.zeros(2), np.zeros(2)
        out = pv3d.Outputs(None, pw.ctypes.data, pr.ctypes.data, en.ctypes.data, None, None, 0)
        p = ctx.params(w.map_n, w.k)
        s = np.ascontiguousarray(w.sweep.sun_xyz, np.float64)
        arr = [np.ascontiguousarray(a, np.float64) for a in (w.sweep.dni, w.sweep.d_poa, w.sweep.dt_h)]
        st = pv3d.lib().pv3d_evaluate_noalloc(ctx.h, sh, gh, s.ctypes.data, arr[0].ctypes.data, arr[1].ctypes.data,
                                              arr[2].ctypes.data, 2, ctypes.byref(p), ctypes.byref(out), None)
        assert st == pv3d.EINVAL
    finally:
        ctx.release_scene(sh)
        ctx.release_generator(gh)
