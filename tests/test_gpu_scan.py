"""The scan of the tile counts on both sides of its register limit (needs an MI355X).

The scan's one workgroup of 512 threads gives each thread a run of tiles. Up
to 8 tiles per thread (at most 4,096 tiles), a thread keeps its counts in
registers for the later passes; above that, it reads them back from memory.
Here the same sweep runs at tile counts on both sides of that limit, with
identical shaded flags and powers, each equal to the oracle's:
- N = 4096 at 64-texel tiles: 4,096 tiles, registers;
- N = 4096 at 32-texel tiles: 16,384 tiles, memory;
- N = 4160 at 64-texel tiles: 4,225 tiles, memory."""
import numpy as np
import pytest

from paper_1410_5780_amd import workloads as W
from tests.test_gpu_parity import ctx, _say  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("map_n,tiles", [(4096, (64, 32, 128)), (4160, (64, 32))])
def test_scan_register_and_memory_paths_agree(ctx, oracle_lib, map_n, tiles):
    w = W.random_tiny(71, n_boxes=10, n_loose=80, n_mod_side=3, map_n=map_n, k=4, n_sun=4)
    sh, gh = ctx.load_scene(w.scene), ctx.define_generator(w.gen)
    try:
        outs = [ctx.evaluate(sh, gh, w.gen, w.sweep, w.map_n, w.k, export_bits=True, tile=t) for t in tiles]
    finally:
        ctx.release_scene(sh)
        ctx.release_generator(gh)
    ref = oracle_lib.evaluate(w.scene, w.gen, w.sweep, w.map_n, w.k)
    for t, o in zip(tiles, outs):
        assert np.array_equal(o.counts, ref.counts), (map_n, t)
        assert np.array_equal(o.bits, outs[0].bits), (map_n, t)
        assert np.array_equal(o.power, ref.power) and np.array_equal(o.energy, ref.energy), (map_n, t)
    _say(f"[scan] N={map_n}, tiles {tiles}: {int(ref.counts.sum())} shaded samples, identical to the oracle")
