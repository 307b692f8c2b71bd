"""Parity at the largest sizes the C ABI accepts (needs an MI355X).

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
