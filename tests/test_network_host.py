"""Host-side logic of the network code (no GPU): the average pool folded
into the next layer's weights (Sec. 3.3) multiplies exactly the window sums
of the unpooled spikes."""
import numpy as np
import pytest

from paper_2309_09025_amd.network import fold_avg_pool


@pytest.mark.parametrize("C,H,W,k", [(10, 12, 12, 2), (2, 4, 4, 2), (3, 5, 7, 2), (2, 6, 6, 3)])
def test_folded_pool_weights_multiply_window_sums(C, H, W, k):
    g = np.random.Generator(np.random.PCG64(C * 100 + H * 10 + k))
    Hp, Wp = H // k, W // k
    W1 = g.integers(-8, 9, size=(5, C * Hp * Wp))
    s = g.integers(0, 3, size=C * H * W)
    blocks = s.reshape(C, H, W)[:, : k * Hp, : k * Wp].reshape(C, Hp, k, Wp, k)
    window_sums = blocks.sum(axis=(2, 4)).reshape(-1)
    folded = fold_avg_pool(W1, C, H, W, k).astype(np.int64)
    assert folded.shape == (5, C * H * W)
    assert np.array_equal(folded @ s, W1 @ window_sums)
