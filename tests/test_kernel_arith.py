"""Integer identities the GPU kernels rely on, checked exhaustively on the CPU.

The tile kernel finds a sample's cell as floor(q / k) with k known only at run
time. It takes the high word of q * m, m = ceil(2^32 / k), instead of a division;
the identity must hold for every sample index q the kernel can meet (below
k * cells per module side, far below 2^32 / k)."""
import numpy as np


def _mulhi_div(q: np.ndarray, k: int) -> np.ndarray:
    if k == 1:
        return q.copy()
    m = np.uint64(((1 << 32) + k - 1) // k)
    return ((q.astype(np.uint64) * m) >> np.uint64(32)).astype(np.int64)


def test_multiply_high_division_is_exact_for_small_indices():
    q = np.arange(1 << 16, dtype=np.int64)
    for k in range(1, 65):
        np.testing.assert_array_equal(_mulhi_div(q, k), q // k, err_msg=f"k={k}")


def test_multiply_high_division_holds_up_to_its_bound():
    # the bound q < 2^32 / k: the last 4,096 indices below it, and a spread of indices across the range
    for k in (2, 3, 5, 7, 8, 10, 12, 16, 31, 64, 100, 255, 256):
        top = ((1 << 32) - 1) // k
        q = np.concatenate([np.arange(max(0, top - 4096), top + 1, dtype=np.int64),
                            np.linspace(0, top, 10001).astype(np.int64)])
        np.testing.assert_array_equal(_mulhi_div(q, k), q // k, err_msg=f"k={k}")
