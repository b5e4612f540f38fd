"""Patch ray batches (mnr_patch_rays): corners from the published SplitMix64
stream (the oracle's generator), each patch a contiguous size x size block
inside the image, deterministic per seed."""
import numpy as np
import pytest

from oracle.rng import splitmix64


def test_patch_batch_layout_and_corners():
    import paper_2306_16541_amd as m
    H, W, n, size, seed = 96, 128, 6, 20, 12345
    ids = m.patch_rays(H, W, n, size, seed)
    assert ids.shape == (n * size * size,)
    assert ids.min() >= 0 and ids.max() < H * W
    for k in range(n):
        p = ids[k * size * size:(k + 1) * size * size].reshape(size, size)
        y0, x0 = divmod(int(p[0, 0]), W)
        assert np.array_equal(p, (y0 + np.arange(size))[:, None] * W + x0 + np.arange(size)[None, :])
        zy, zx = (int(v) for v in splitmix64(seed, [2 * k, 2 * k + 1]))
        assert y0 == ((zy >> 11) * (H - size + 1)) >> 53
        assert x0 == ((zx >> 11) * (W - size + 1)) >> 53
    assert np.array_equal(ids, m.patch_rays(H, W, n, size, seed))
    assert not np.array_equal(ids, m.patch_rays(H, W, n, size, seed + 1))


def test_patch_that_does_not_fit_is_rejected():
    import paper_2306_16541_amd as m
    with pytest.raises(m.MnrError, match="fit"):
        m.patch_rays(16, 16, 2, 20, 0)
