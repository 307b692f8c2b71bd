"""Parity at the largest sizes the C ABI accepts, and for degenerate suns (needs an MI355X).

- **N = 16384**, the largest depth picture. The full pictures are exported
  and compared texel by texel: 2 suns of 268 M texels.
- **k = 255**, the most samples per cell: 65,025 per cell, with k * n_cv =
  2,550 within the 4,095 limit. Every 64-texel tile then holds far more
  samples than a rect of the sparse route takes, so rects split down to 16
  texels, and the densest fall back to the full route.

Shaded flags, counts and depth pictures must be bit-identical to the
oracle's, and powers must agree within the path's tolerance."""
import pytest

from paper_1410_5780_amd import workloads as W
from tests.test_gpu_parity import compare, ctx  # noqa: F401  (fixture)

pytestmark = pytest.mark.gpu


def test_largest_depth_picture(ctx, oracle_lib):
    w = W.random_tiny(81, n_boxes=6, n_loose=40, n_mod_side=3, map_n=16384, k=8, n_sun=2)
    got, ref = compare(ctx, oracle_lib, w, maps=True, bits=True)
    assert ref.counts.sum() > 1000


def test_most_samples_per_cell(ctx, oracle_lib):
    w = W.random_tiny(81, n_boxes=6, n_loose=6, n_mod_side=2, map_n=256, k=255, n_sun=2)
    assert w.k * w.gen.n_cv <= 4095 and w.k * w.gen.n_cu <= 4095
    got, ref = compare(ctx, oracle_lib, w, maps=True, bits=True)
    assert ref.counts.sum() > 100000


def test_zenith_sun_horizon_sun_and_basis_switch(ctx, oracle_lib):
    """Degenerate suns over a horizontal generator:
    - exactly at the zenith: every box wall is edge-on, with no area in the picture, and the sun
      lies along the modules' normal;
    - exactly on the horizon: not up, so every output is zero;
    - either side of the image basis switch (|d_z| = 0.9 and a hair below): both sides take the same
      branch from the same input."""
    import numpy as np
    w = W.random_tiny(91, n_boxes=8, n_loose=10, n_mod_side=3, tilt_deg=0.0, map_n=256, k=4, n_sun=1)
    a, b = np.sqrt(1.0 - 0.9 ** 2), 0.9 - 1e-9
    dirs = np.array([[0.0, 0.0, 1.0], [1.0, 0.0, 0.0], [a, 0.0, 0.9], [np.sqrt(1.0 - b * b), 0.0, b]])
    n = len(dirs)
    sw = W.Sweep(dirs, np.full(n, 800.0), np.full(n, 50.0), np.ones(n), np.zeros(n, np.int32), np.zeros(n))
    got, ref = compare(ctx, oracle_lib, W.Workload("degenerate_suns", w.scene, w.gen, sw, 256, 4))
    assert got.counts[0].sum() > 0 and got.counts[2].sum() > 0
    assert got.counts[1].sum() == 0 and got.power[1] == 0.0 and got.power_ref[1] == 0.0


@pytest.mark.parametrize("n_cu,n_cv", [(4095, 1), (1, 4095)])
def test_most_cells_per_module_side(ctx, oracle_lib, n_cu, n_cv):
    """4,095 cells along one module side at k = 1, the most the ABI takes: a module has more cells
    than the tile kernel's per-wave LDS cell counters, so counts go to device memory directly."""
    import dataclasses
    import numpy as np
    base = W.random_tiny(94, n_boxes=8, n_loose=30, n_mod_side=2, map_n=512, k=1, n_sun=4)
    g = dataclasses.replace(base.gen, n_cu=n_cu, n_cv=n_cv, n_sub=3,
                            cell_substring=(np.arange(n_cu * n_cv) % 3).astype(np.int32))
    got, ref = compare(ctx, oracle_lib, W.Workload(f"cells_{n_cu}x{n_cv}", base.scene, g, base.sweep, 512, 1))
    assert ref.counts.sum() > 1000
